"""Bit-exact parity of the gfx950 path against the CPU oracle (needs a GPU).

Every case calls the C ABI (through the ctypes binding) on seeded synthetic
Bernoulli(0.5) blocks and compares the packed output with the oracle word
for word.  Every block, up to the largest supported transform length, is compared in
full; the 12.8e6-bit block is also checked for linearity in the key.
"""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def gpu_hash(key, n, seed, m):
    out = pa.toeplitz_hash(dev(key), n, dev(seed), m)
    return host(out)[: wl.words(m)]


def check_full(n, m, cfg=10, idx=0, garbage=False):
    key, seed = wl.key_and_seed(cfg, n, m, idx, garbage_tail=garbage)
    got = gpu_hash(key, n, seed, m)
    want = oracle.toeplitz_hash(key, n, seed, m)
    assert np.array_equal(got, want), "n=%d m=%d: %d words differ" % (n, m, int(np.sum(got != want)))
    return key, seed, got


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True, scope="module")
def _gpu():
    require_gpu()
    oracle.build()
    yield


EDGE = [(1, 1), (2, 1), (2, 2), (63, 1), (64, 64), (65, 65), (65, 1), (127, 64), (128, 128), (129, 1),
        (1000, 1), (1000, 999), (1000, 1000), (4095, 1), (4096, 1), (4097, 2048), (4033, 64), (4034, 64),
        (3000, 1000), (5000, 2500), (4609, 4608)]


@pytest.mark.parametrize("n,m", EDGE)
def test_edge_shapes(n, m):
    check_full(n, m, cfg=11, idx=n * 7 + m)


@pytest.mark.parametrize("n,m", [(262_144, 65_536), (100_003, 31_337), (65_536, 65_536), (300_000, 27_001)])
def test_multi_tile_ragged(n, m):
    check_full(n, m, cfg=12)


def test_garbage_padding_is_ignored():
    n, m = 100_001, 20_003
    k1, s1, y1 = check_full(n, m, cfg=13, garbage=False)
    _, _, y2 = check_full(n, m, cfg=13, garbage=True)
    assert np.array_equal(y1, y2)


def test_length_boundaries():
    # shapes whose required length sits exactly on / just past supported lengths
    for L in [4096, 4608, 6144, 8192, 3 * 2**17, 2**18]:
        m = 64
        n_exact = L - 64 + 1          # required_len = (n-1 rounded to 64) + 64 = L
        assert pa.transform_len(n_exact, m) == L and pa.transform_len(n_exact + 1, m) > L
        for n in (n_exact, n_exact + 1):
            check_full(n, m, cfg=14, idx=n)


def test_paper_finite_size_block():
    # n = 10^6, m = 250,000 (Sec. 2.1: blocks of at least 10^6 bits), full oracle
    check_full(1_000_000, 250_000, cfg=2)


def test_large_block_full_and_linear():
    # n = 12.8e6, m = 1.28e6: every output word against the oracle, plus
    # linearity in the key (a property that holds at any size)
    n, m = 12_800_000, 1_280_000
    key, seed = wl.key_and_seed(3, n, m, 0)
    key2 = wl.random_bits(n, wl.rng(3, wl.ROLE_KEY, 1))
    y = gpu_hash(key, n, seed, m)
    want = oracle.toeplitz_hash(key, n, seed, m)
    assert np.array_equal(y, want), "%d of %d words differ" % (int(np.sum(y != want)), want.size)
    y2 = gpu_hash(key2, n, seed, m)
    y12 = gpu_hash(key ^ key2, n, seed, m)
    assert np.array_equal(y12, y ^ y2), "linearity in the key"


def test_largest_supported_block_full():
    # the largest transform length (27 * 2^20): the row pass cannot hold two
    # rows in LDS, so the seed spectrum goes through HBM (P2 modes 1 and 0)
    n, m = 24_000_000, 4_300_000
    assert pa.transform_len(n, m) == 27 * 2**20
    key, seed = wl.key_and_seed(15, n, m, 0)
    y = gpu_hash(key, n, seed, m)
    want = oracle.toeplitz_hash(key, n, seed, m)
    assert np.array_equal(y, want), "%d of %d words differ" % (int(np.sum(y != want)), want.size)


def test_all_ones_extremes():
    # c[k] reaches n (largest convolution value) with all-ones key and seed
    n, m = 200_000, 50_000
    key = np.full(wl.words(n), np.uint64(2**64 - 1), dtype=np.uint64)
    seed = np.full(wl.words(n + m - 1), np.uint64(2**64 - 1), dtype=np.uint64)
    got = gpu_hash(key, n, seed, m)
    want = oracle.toeplitz_hash(key, n, seed, m)
    assert np.array_equal(got, want)


def test_plan_matches_plain_and_is_length_invariant():
    S = 400_000
    seed = wl.random_bits(S, wl.rng(16, wl.ROLE_SEED, 0))
    dseed = dev(seed)
    shapes = [(300_000, 99_999), (200_000, 50_000), (1000, 1000), (399_000, 1001)]
    with pa.Plan(dseed, S) as plan, pa.Plan(dseed, S, transform_len=2**20) as big:
        assert big.transform_len == 2**20 and plan.transform_len < 2**20
        for i, (n, m) in enumerate(shapes):
            key = wl.random_bits(n, wl.rng(16, wl.ROLE_KEY, i))
            want = oracle.toeplitz_hash(key, n, seed, m)
            a = host(plan.hash(dev(key), n, m))[: wl.words(m)]
            b = host(big.hash(dev(key), n, m))[: wl.words(m)]
            assert np.array_equal(a, want) and np.array_equal(b, want), (n, m)
        with pytest.raises(pa.PAError):
            plan.hash(dev(wl.random_bits(S, wl.rng(16, 1, 9))), S, 2)


def test_batched_matches_oracle():
    shapes = [(262_144, 13_000), (100_000, 50_000), (4096, 1), (777_777, 200_001), (65, 65), (300_001, 30_001)]
    blocks, refs = [], []
    shared_seed = None
    for i, (n, m) in enumerate(shapes):
        key, seed = wl.key_and_seed(17, n, m, i)
        if i == 5:  # reuse an earlier seed buffer (shared seeds are allowed)
            seed = shared_seed
        if i == 3:
            shared_seed = seed
        blocks.append((dev(key), n, dev(seed), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
        refs.append(oracle.toeplitz_hash(key, n, seed, m))
    outs = pa.toeplitz_hash_batched(blocks)
    for o, r in zip(outs, refs):
        assert np.array_equal(host(o)[: r.size], r)


def test_deterministic_repeats():
    n, m = 300_000, 70_000
    key, seed = wl.key_and_seed(18, n, m, 0)
    dk, ds = dev(key), dev(seed)
    first = host(pa.toeplitz_hash(dk, n, ds, m))
    outs = [pa.toeplitz_hash(dk, n, ds, m) for _ in range(100)]
    for o in outs:
        assert np.array_equal(host(o), first)


def test_stream_ordering_on_side_stream():
    n, m = 500_000, 100_000
    key, seed = wl.key_and_seed(19, n, m, 0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dk, ds = dev(key), dev(seed)
        out = pa.toeplitz_hash(dk, n, ds, m, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64)[: wl.words(m)], oracle.toeplitz_hash(key, n, seed, m))


def test_batched_uneven_blocks_match_single_calls_and_oracle():
    # log-uniform n in [2^14, 2^19], m/n in [0.05, 0.5]: many length classes
    g = np.random.default_rng(21)
    blocks, keys = [], []
    for i in range(40):
        n = int(round(2.0 ** g.uniform(14, 19)))
        m = max(1, int(round(n * g.uniform(0.05, 0.5))))
        key, seed = wl.key_and_seed(22, n, m, i)
        keys.append((key, seed, n, m))
        blocks.append((dev(key), n, dev(seed), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
    assert len({pa.transform_len(n, m) for _, _, n, m in keys}) >= 5
    outs = pa.toeplitz_hash_batched(blocks)
    order = list(range(len(blocks)))[::-1]  # permuted submission gives the same per-block results
    outs2 = pa.toeplitz_hash_batched([(blocks[i][0], blocks[i][1], blocks[i][2], blocks[i][3],
                                       torch.zeros_like(blocks[i][4])) for i in order])
    for j, i in enumerate(order):
        key, seed, n, m = keys[i]
        want = oracle.toeplitz_hash(key, n, seed, m)
        assert np.array_equal(host(outs[i])[: want.size], want), (i, n, m)
        assert np.array_equal(host(outs2[j])[: want.size], want)
        if i % 8 == 0:
            assert np.array_equal(gpu_hash(key, n, seed, m), want)


def test_batched_groups_join_back_into_the_callers_stream():
    # length groups run on side lanes; the outputs must be complete for work
    # queued afterwards on the caller's stream (only that stream is synced)
    g = np.random.default_rng(24)
    shapes = [(2_000_000, 500_000)] + [(int(round(2.0 ** g.uniform(13, 17))), 0) for _ in range(11)]
    blocks, keys = [], []
    for i, (n, m) in enumerate(shapes):
        m = m or max(1, n // 5)
        key, seed = wl.key_and_seed(25, n, m, i)
        keys.append((key, seed, n, m))
        blocks.append((dev(key), n, dev(seed), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
    assert len({pa.transform_len(n, m) for _, _, n, m in keys}) >= 4
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for b in blocks:
            b[4].record_stream(s)
        for rep in range(2):
            pa.toeplitz_hash_batched(blocks, stream=s)
            copies = [b[4].clone() for b in blocks]   # queued on s after the call
            s.synchronize()
            for i, (key, seed, n, m) in enumerate(keys):
                if n > 1_000_000:
                    idx = np.arange(0, m, 997)
                    words_ = copies[i].cpu().numpy().view(np.uint64)
                    got = ((words_[idx >> 6] >> (idx & 63).astype(np.uint64)) & np.uint64(1)).astype(np.uint8)
                    assert np.array_equal(got, oracle.toeplitz_bits(key, n, seed, m, idx)), (rep, i)
                else:
                    want = oracle.toeplitz_hash(key, n, seed, m)
                    assert np.array_equal(copies[i].cpu().numpy().view(np.uint64)[: want.size], want), (rep, i)
            for b in blocks:
                b[4].zero_()


def _shape_for(L, ratio=0.25):
    n = int(L * 0.79) // 64 * 64
    while pa.transform_len(n, max(1, int(n * ratio))) != L:
        n -= 64
    return n, max(1, int(n * ratio))


@pytest.mark.parametrize("k", [8, 9, 10, 12, 13])
def test_lengths_with_27_split_first_rounds(k):
    # 27 | C: the row transform starts with a 9-value round, then a round
    # holding the last radix-3 stage (the first round's stride is 3 * 2^j)
    L = 27 * 2**k
    info = pa.plan_info(L)
    assert info["row_round_size"][0] == 9 and info["row_round_size"][1] in (3, 6)
    n, m = _shape_for(L)
    key, seed = wl.key_and_seed(26, n, m, k)
    want = oracle.toeplitz_hash(key, n, seed, m)
    assert np.array_equal(gpu_hash(key, n, seed, m), want)
    with pa.Plan(dev(seed), n + m - 1, transform_len=L) as plan:     # seed-spectrum and plan passes
        assert np.array_equal(host(plan.hash(dev(key), n, m))[: want.size], want)


def test_profile_records_every_kernel():
    n, m = 300_000, 60_000
    key, seed = wl.key_and_seed(23, n, m, 0)
    dk, ds = dev(key), dev(seed)
    pa.profile_enable(True)
    try:
        for _ in range(3):
            pa.toeplitz_hash(dk, n, ds, m)
        torch.cuda.synchronize()
        prof = pa.profile_collect()
    finally:
        pa.profile_enable(False)
    assert set(prof) >= {"colfwd", "rowconv", "colinv"}
    for st in prof.values():
        assert st["launches"] == 3 and st["avg_ms"] > 0 and st["alg_bytes"] > 0 and st["alg_ops"] > 0
    assert pa.profile_collect() == {}


def test_alu_probe_rates_are_plausible():
    r = pa.alu_probe()
    # an FMA rate within reach of the 39.3 T/s issue peak, and a modular
    # product costing about three FMAs
    assert 5.0 < r["fma_Tops"] < 45.0
    assert 0.15 < r["mulmod_Gops"] * 1e-3 / r["fma_Tops"] < 0.5


def test_launch_and_phase_probes():
    # an empty launch costs a few microseconds; the phase probe checks the
    # two forms of its three phases against each other before timing them
    us = pa.launch_probe(256, 768, reps=100)
    assert 0.2 < us < 100.0
    r = pa.phase_probe()
    assert r["workgroups"] >= 1 and r["threads"] == 768 and r["tiles"] == 8 * r["workgroups"]
    for k in ("empty_launch_us", "empty_cooperative_us", "three_launches_us", "cooperative_grid_sync_us",
              "tiles_no_release_us", "tiles_release_us"):
        assert 0.0 < r[k] < 10_000.0, k
    with pytest.raises(pa.PAError):
        pa.launch_probe(1, 100)
