"""Serving loop on the GPU: every served result equals the same request run
alone (pa_toeplitz_hash), a sample matches the CPU oracle, the budget holds,
and requests overlap on the device."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def test_served_results_equal_alone_and_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = np.random.default_rng(31)
    seeds = [wl.random_bits(L, wl.rng(30, wl.ROLE_SEED, i)) for i, L in enumerate([3_000_000, 1_200_000])]
    dseeds = [dev(s) for s in seeds]
    reqs = []
    for i in range(60):
        sid = int(g.integers(0, 2))
        n = int(round(10 ** g.uniform(4.5, 6.2)))
        n = min(n, 700_000 if sid == 1 else 2_000_000)
        m = max(1, min(n, int(round(n * g.uniform(0.1, 0.5)))))
        key = wl.random_bits(n, wl.rng(30, wl.ROLE_KEY, i))
        reqs.append((sid, key, n, m))
    budget = 64 << 20  # a handful of requests at a time
    with pa.Server(budget, max_inflight=16, streams=3) as srv:
        ids = [srv.register_seed(dseeds[k], seeds[k].size * 64) for k in range(2)]
        outs, tickets, keep = [], [], []
        for sid, key, n, m in reqs:
            keep.append(dev(key))
            outs.append(torch.zeros(wl.words(m), dtype=torch.int64, device="cuda"))
        # the server's streams are not ordered after torch's: inputs must be
        # complete, and no zero-fill pending, before the requests go in
        torch.cuda.synchronize()
        for (sid, key, n, m), dk, out in zip(reqs, keep, outs):
            tickets.append(srv.submit(ids[sid], dk, n, m, out))
        srv.drain()
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["peak_bytes_in_flight"] <= budget
        assert st["peak_inflight"] >= 2 and st["batches"] >= 3
        lat = [srv.latency_us(t) for t in tickets]
        assert min(lat) > 0
    torch.cuda.synchronize()
    for i, ((sid, key, n, m), out) in enumerate(zip(reqs, outs)):
        served = out.cpu().numpy().view(np.uint64)[: wl.words(m)]
        alone = pa.toeplitz_hash(keep[i], n, dseeds[sid], m)
        torch.cuda.synchronize()
        assert np.array_equal(served, alone.cpu().numpy().view(np.uint64)[: wl.words(m)]), i
        if i % 10 == 0:
            assert np.array_equal(served, oracle.toeplitz_hash(key, n, seeds[sid], m)), i


def test_small_request_does_not_wait_for_a_large_one():
    """A small request submitted right after a large one completes first,
    whether the scheduler batches the two together (each length group
    completes on its own event) or not (the batch goes to a free stream)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n_big, m_big = 8_000_000, 2_000_000
    n_small, m_small = 50_000, 10_000
    seed = wl.random_bits(n_big + m_big, wl.rng(32, wl.ROLE_SEED, 0))
    dseed = dev(seed)
    pairs = []
    with pa.Server(1 << 30, max_inflight=64, streams=2) as srv:
        sid = srv.register_seed(dseed, seed.size * 64)
        for i in range(6):
            kb = dev(wl.random_bits(n_big, wl.rng(32, wl.ROLE_KEY, 2 * i)))
            ks = dev(wl.random_bits(n_small, wl.rng(32, wl.ROLE_KEY, 2 * i + 1)))
            ob = torch.zeros(wl.words(m_big), dtype=torch.int64, device="cuda")
            os_ = torch.zeros(wl.words(m_small), dtype=torch.int64, device="cuda")
            torch.cuda.current_stream().synchronize()   # inputs complete before the server's streams read them
            tb = srv.submit(sid, kb, n_big, m_big, ob)
            ts = srv.submit(sid, ks, n_small, m_small, os_)
            pairs.append((tb, ts, kb, ks, ob, os_))
            srv.drain()
        for tb, ts, *_ in pairs:
            # submitted later and finished sooner: completed first
            assert srv.latency_us(ts) < srv.latency_us(tb)
    torch.cuda.synchronize()
    for _, _, kb, ks, ob, os_ in pairs:
        assert torch.equal(ob, pa.toeplitz_hash(kb, n_big, dseed, m_big))
        assert torch.equal(os_, pa.toeplitz_hash(ks, n_small, dseed, m_small))


def test_spectra_built_on_demand_evicted_and_rebuilt_under_a_small_budget():
    """A budget that holds few spectra: every (seed, length) pair is built
    on first use on the server's build stream (requests wait on the device,
    not the scheduler), unused spectra are evicted and rebuilt when needed
    again, and seeds registered while requests run are served too.  Every
    result equals the same request run alone."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n_seeds = 6
    seeds = [wl.random_bits(1_500_000, wl.rng(33, wl.ROLE_SEED, i)) for i in range(n_seeds)]
    dseeds = [dev(sd) for sd in seeds]
    g = np.random.default_rng(34)
    with pa.Server(48 << 20, max_inflight=32, streams=3) as srv:
        ids = [srv.register_seed(dseeds[k], 1_500_000) for k in range(3)]
        reqs, outs, keys = [], [], []
        for i in range(90):
            if i == 30:   # registered while earlier requests are on the device
                ids += [srv.register_seed(dseeds[k], 1_500_000) for k in range(3, n_seeds)]
            sid = int(g.integers(0, len(ids)))
            n = int(round(10 ** g.uniform(4.5, 6.0)))
            m = max(1, min(n, int(round(n * g.uniform(0.1, 0.5)))))
            key = dev(wl.random_bits(n, wl.rng(33, wl.ROLE_KEY, i)))
            out = torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")
            keys.append(key)
            outs.append(out)
            # torch's stream only: earlier requests stay on the device
            torch.cuda.current_stream().synchronize()
            reqs.append((sid, n, m, srv.submit(ids[sid], key, n, m, out)))
        srv.drain()
        st = srv.stats()
        assert st["completed"] == 90 and st["failed"] == 0
        assert st["spectra_evicted"] > 0 and st["spectra_built"] > st["spectra_resident"]
        assert st["peak_bytes_in_flight"] <= 48 << 20
    torch.cuda.synchronize()
    for (sid, n, m, _), key, out in zip(reqs, keys, outs):
        alone = pa.toeplitz_hash(key, n, dseeds[sid], m)
        torch.cuda.synchronize()
        assert torch.equal(out[: wl.words(m)], alone[: wl.words(m)]), (sid, n, m)
