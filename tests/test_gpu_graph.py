"""Graph form of the batched call on the GPU: a captured launch sequence
over fixed buffers, replayed several times with new key contents, eager
work and synchronizations between replays; every replay is compared with
the eager batched call and with the CPU oracle."""
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
    return t.cpu().numpy().view(np.uint64)[: wl.words(m)]


@pytest.fixture(autouse=True, scope="module")
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    yield


def _shapes(seed, count, lo, hi, modified):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(2.0 ** g.uniform(lo, hi)))
        m = max(1, int(round(n * g.uniform(0.05, 0.5))))
        if modified:
            m = min(m, n - 1)
        out.append((n, m))
    return out


@pytest.mark.parametrize("modified", [False, True])
def test_replays_follow_buffer_contents(modified):
    shapes = _shapes(60 + modified, 14, 12, 19, modified)
    assert len({pa.transform_len(n - m if modified else n, m) for n, m in shapes}) >= 4
    seeds = [wl.random_bits(n - 1 if modified else n + m - 1, wl.rng(61, wl.ROLE_SEED, i))
             for i, (n, m) in enumerate(shapes)]
    keys = [dev(np.zeros(wl.words(n), np.uint64)) for n, _ in shapes]
    dseeds = [dev(s) for s in seeds]
    outs = [torch.zeros(wl.words(m), dtype=torch.int64, device="cuda") for _, m in shapes]
    blocks = [(keys[i], n, dseeds[i], m, outs[i]) for i, (n, m) in enumerate(shapes)]
    eager_outs = [torch.zeros_like(o) for o in outs]
    eager_blocks = [(keys[i], n, dseeds[i], m, eager_outs[i]) for i, (n, m) in enumerate(shapes)]
    ref = pa.modified_toeplitz_hash_batched if modified else pa.toeplitz_hash_batched
    fn = oracle.modified_toeplitz_hash if modified else oracle.toeplitz_hash
    with pa.BatchGraph(blocks, modified=modified) as g:
        assert g.block_count == len(shapes)
        for rep in range(4):
            # new key contents, written in place (the graph keeps the pointers)
            host_keys = [wl.random_bits(n, wl.rng(62, wl.ROLE_KEY, 100 * rep + i)) for i, (n, _) in enumerate(shapes)]
            for k, hk in zip(keys, host_keys):
                k.copy_(dev(hk))
            for o in outs:
                o.fill_(-1)
            torch.cuda.synchronize()
            g.launch()
            ref(eager_blocks)                      # eager work between replays, same stream
            torch.cuda.synchronize()
            for i, (n, m) in enumerate(shapes):
                got = host(outs[i], m)
                assert np.array_equal(got, host(eager_outs[i], m)), (rep, i, n, m)
                if i % 4 == rep % 4:
                    assert np.array_equal(got, fn(host_keys[i], n, seeds[i], m)), (rep, i, n, m)


def test_replay_on_a_side_stream_and_recreate():
    shapes = _shapes(63, 6, 14, 18, False)
    ins = [wl.key_and_seed(64, n, m, i) for i, (n, m) in enumerate(shapes)]
    blocks = [(dev(k), n, dev(s), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda"))
              for (k, s), (n, m) in zip(ins, shapes)]
    want = [oracle.toeplitz_hash(k, n, s, m) for (k, s), (n, m) in zip(ins, shapes)]
    st = torch.cuda.Stream()
    for _ in range(2):
        g = pa.BatchGraph(blocks)
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            for _ in range(3):
                g.launch(stream=st)
            copies = [b[4].clone() for b in blocks]   # ordered after the replays on st
        st.synchronize()
        for i, (n, m) in enumerate(shapes):
            assert np.array_equal(host(copies[i], m), want[i]), i
        g.destroy()
        for b in blocks:
            b[4].zero_()
        torch.cuda.synchronize()


def test_update_points_the_graph_at_new_buffers():
    shapes = _shapes(65, 8, 13, 17, False)
    def make(cfg):
        ins = [wl.key_and_seed(cfg, n, m, i) for i, (n, m) in enumerate(shapes)]
        bl = [(dev(k), n, dev(s), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda"))
              for (k, s), (n, m) in zip(ins, shapes)]
        return ins, bl
    ins1, bl1 = make(66)
    ins2, bl2 = make(67)
    with pa.BatchGraph(bl1) as g:
        g.launch()
        g.update(bl2)             # same shapes, other buffers
        g.launch()
        torch.cuda.synchronize()
        for (k, s), (n, m), b in zip(ins2, shapes, bl2):
            assert np.array_equal(host(b[4], m), oracle.toeplitz_hash(k, n, s, m))
        for (k, s), (n, m), b in zip(ins1, shapes, bl1):
            assert np.array_equal(host(b[4], m), oracle.toeplitz_hash(k, n, s, m))
        # reordered blocks form the same groups; a different length does not
        g.update(bl1[::-1])
        g.launch()
        torch.cuda.synchronize()
        for (k, s), (n, m), b in zip(ins1, shapes, bl1):
            assert np.array_equal(host(b[4], m), oracle.toeplitz_hash(k, n, s, m))
        n0, m0 = shapes[0]
        k0, s0 = wl.key_and_seed(68, 4 * n0, m0, 0)
        bad = [(dev(k0), 4 * n0, dev(s0), m0, torch.zeros(wl.words(m0), dtype=torch.int64, device="cuda"))] + bl1[1:]
        with pytest.raises(pa.PAError):
            g.update(bad)
        with pytest.raises(pa.PAError):
            g.update(bl1[:-1])
