"""Geometry tuning on the GPU: every valid R x C split of a length gives the
same bits (the four-step split of Sec. 3.1 is a free choice), the autotuner
installs a valid split, and plans and server spectra built before a change
of the table keep working."""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, M = 100_003, 25_001


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host(t, m):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)[: wl.words(m)]


def valid_splits(L):
    out = []
    for a in range(1, 11):
        for w in (16, 32, 64):
            try:
                pa.plan_info(L, a, w)
            except pa.PAError:
                continue
            out.append((a, w))
    return out


@pytest.fixture(autouse=True)
def _gpu_and_restore():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    yield
    L = pa.transform_len(N, M)
    for cls in (0, 1):
        pa.tune_set(L, cls, 0, 0)


def test_every_split_gives_the_same_bits():
    key, seed = wl.key_and_seed(40, N, M, 0)
    want = oracle.toeplitz_hash(key, N, seed, M)
    L = pa.transform_len(N, M)
    splits = valid_splits(L)
    assert len(splits) >= 6
    dk, ds = dev(key), dev(seed)
    blocks_np = [wl.key_and_seed(41, N, M, i) for i in range(3)]
    blocks_want = [oracle.toeplitz_hash(k, N, s, M) for k, s in blocks_np]
    bdev = [(dev(k), dev(s)) for k, s in blocks_np]
    for a, w in splits:
        print("split log2_rows=%d tile_width=%d" % (a, w), flush=True)
        pa.tune_set(L, 0, a, w)
        assert pa.tune_get(L, 0) == (a, w)
        got = host(pa.toeplitz_hash(dk, N, ds, M), M)
        assert np.array_equal(got, want), (a, w)
        pa.tune_set(L, 1, a, w)
        outs = [torch.zeros(wl.words(M), dtype=torch.int64, device="cuda") for _ in bdev]
        pa.toeplitz_hash_batched([(k, N, s, M, o) for (k, s), o in zip(bdev, outs)])
        for i, o in enumerate(outs):
            assert np.array_equal(host(o, M), blocks_want[i]), (a, w, i)


@pytest.mark.parametrize("count", [1, 4])
def test_autotune_installs_a_valid_split(count):
    L = pa.transform_len(N, M)
    r = pa.autotune(L, count=count, reps=2)
    cls = 0 if count == 1 else 1
    # every split, then row round splits and row workgroup sizes
    assert r["candidates"] >= len(valid_splits(L)) + 4
    g = pa.tune_get_geometry(L, cls)
    assert (g["log2_rows"], g["tile_width"], g["row_first"], g["row_threads"]) == (
        r["log2_rows"], r["tile_width"], r["row_first"], r["row_threads"])
    assert 0 < r["best_us"] <= r["default_us"]
    key, seed = wl.key_and_seed(42, N, M, count)
    got = host(pa.toeplitz_hash(dev(key), N, dev(seed), M), M)
    assert np.array_equal(got, oracle.toeplitz_hash(key, N, seed, M))


def test_autotune_rejects_bad_arguments():
    L = pa.transform_len(N, M)
    for args in [(L, 0, 2), (L, 1, 0), (L + 1, 1, 2), (2**24 * 3, 4096, 1)]:
        with pytest.raises(pa.PAError):
            pa.autotune(*args)


def test_plan_and_server_keep_their_geometry_across_a_table_change():
    L = pa.transform_len(N, M)
    splits = valid_splits(L)
    first, second = splits[0], splits[-1]
    seed_bits = 400_000
    seed = wl.random_bits(seed_bits, wl.rng(43, wl.ROLE_SEED, 0))
    ds = dev(seed)
    keys = [wl.random_bits(N, wl.rng(43, wl.ROLE_KEY, i)) for i in range(6)]
    dkeys = [dev(k) for k in keys]
    want = [oracle.toeplitz_hash(k, N, seed, M) for k in keys]

    pa.tune_set(L, 0, *first)
    with pa.Plan(ds, seed_bits, transform_len=L) as plan:
        pa.tune_set(L, 0, *second)
        assert np.array_equal(host(plan.hash(dkeys[0], N, M), M), want[0])

    pa.tune_set(L, 1, *first)
    with pa.Server(256 << 20, max_inflight=8, streams=2) as srv:
        sid = srv.register_seed(ds, seed_bits)
        outs = [torch.zeros(wl.words(M), dtype=torch.int64, device="cuda") for _ in keys]
        for i in range(3):
            srv.submit(sid, dkeys[i], N, M, outs[i])
        srv.drain()
        pa.tune_set(L, 1, *second)        # the resident spectrum keeps the first split
        for i in range(3, 6):
            srv.submit(sid, dkeys[i], N, M, outs[i])
        srv.drain()
    for i in range(6):
        assert np.array_equal(host(outs[i], M), want[i]), i


@pytest.mark.parametrize("n,m", [(100_003, 25_001), (600_001, 150_001)])
def test_every_row_split_and_row_workgroup_size_gives_the_same_bits(n, m):
    # 100,003 bits: rows of 2^k columns (first round 2, 4 or 8 values);
    # 600,001 bits: rows with a radix-3 stage (first round 3, 6 or 12 values)
    key, seed = wl.key_and_seed(44, n, m, 0)
    want = oracle.toeplitz_hash(key, n, seed, m)
    L = pa.transform_len(n, m)
    a, w = pa.tune_get(L, 0)
    dk, ds = dev(key), dev(seed)
    tried = 0
    for rf in range(0, 5):
        for rt in (0, 256, 512, 768, 1024):
            try:
                pa.tune_set(L, 0, a, w, row_first=rf, row_threads=rt)
            except pa.PAError:
                continue
            tried += 1
            got = host(pa.toeplitz_hash(dk, n, ds, m), m)
            assert np.array_equal(got, want), (rf, rt)
    assert tried >= 12
    pa.tune_set(L, 0, 0, 0)


def test_tune_cache_file_is_written_and_read(tmp_path):
    import subprocess
    import sys
    L = pa.transform_len(N, M)
    path = str(tmp_path / "cache.txt")
    pa.tune_set(L, 1, 0, 0)
    pa.tune_set(2**20, 0, 9, 32)   # an entry the file must carry (autotune may keep the default)
    import os
    old = os.environ.get("PA_TUNE_CACHE")
    os.environ["PA_TUNE_CACHE"] = path
    try:
        pa.autotune(L, count=2, reps=1)
    finally:
        pa.tune_set(2**20, 0, 0, 0)
        if old is None:
            os.environ.pop("PA_TUNE_CACHE", None)
        else:
            os.environ["PA_TUNE_CACHE"] = old
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    assert any(r[:6] == [str(2**20), "0", "9", "32", "0", "0"] for r in rows)
    assert all(len(r) == 7 and r[6].startswith("gfx") for r in rows)
    # write a distinctive geometry for class 1 into the cache and read it
    # back in a fresh process, whose first hash loads the file
    with open(path, "w") as f:
        f.write("%d 1 7 32 0 512 %s\n" % (L, rows[0][6]))
    code = ("import numpy as np, torch, paper_1809_07592_amd as pa\n"
            "k = torch.zeros(%d, dtype=torch.int64, device='cuda'); s = torch.zeros(%d, dtype=torch.int64, device='cuda')\n"
            "pa.toeplitz_hash(k, %d, s, %d); torch.cuda.synchronize()\n"
            "print(pa.tune_get_geometry(%d, 1))\n" % ((N + 63) // 64, (N + M + 62) // 64, N, M, L))
    env = dict(os.environ, PA_TUNE_CACHE=path)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "'log2_rows': 7, 'tile_width': 32, 'row_first': 0, 'row_threads': 512" in out.stdout


def test_tune_cache_is_read_before_queries_and_kept_by_autotune(tmp_path):
    # a fresh process: a query before any hash already sees the file's row,
    # a setting made afterwards wins over the file, and an autotune of
    # another length rewrites the file with the rows it did not tune
    import os
    import subprocess
    import sys
    L = pa.transform_len(N, M)
    path = str(tmp_path / "cache.txt")
    with open(path, "w") as f:
        f.write("%d 1 7 32 0 512 gfx950\n%d 0 9 32 0 0 gfx950\n" % (L, 2**20))
    code = ("import paper_1809_07592_amd as pa\n"
            "print('q', pa.tune_get_geometry(%d, 1))\n"
            "pa.tune_set(%d, 0, 8, 16)\n"
            "print('s', pa.tune_get_geometry(%d, 0))\n"
            "pa.autotune(%d, count=1, reps=1)\n" % (L, 2**20, 2**20, 2**12))
    env = dict(os.environ, PA_TUNE_CACHE=path)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "q {'log2_rows': 7, 'tile_width': 32, 'row_first': 0, 'row_threads': 512}" in out.stdout
    assert "s {'log2_rows': 8, 'tile_width': 16," in out.stdout
    rows = [ln.split()[:6] for ln in open(path) if not ln.startswith("#")]
    assert [str(L), "1", "7", "32", "0", "512"] in rows
    assert [str(2**20), "0", "8", "16", "0", "0"] in rows
    assert any(r[0] == str(2**12) for r in rows) or len(rows) == 2
