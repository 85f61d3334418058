"""Kernels compiled for fixed transform shapes, against the oracle.

The row kernel and the two column kernels have forms compiled for the row
and column transforms of the default geometries of every length from 2^16
up.  Each fixed shape runs here at the smallest length that
uses it, on the plain path (seed and key rows in one row kernel), the plan
path (key row against a resident spectrum, after the spectrum-building mode
of the same kernel) and a batched call, and must give the oracle's bits
(Sec. 2.3 Eq. (4): the product of the Toeplitz matrix and the key).  The
same length under a geometry that no fixed kernel covers runs the general
kernels and must give the same bits.
"""
import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def shape_lengths():
    """Smallest supported length per fixed row shape and per fixed column
    shape (default geometry), as (L, row shape, column shape)."""
    lens = set()
    seen_row, seen_col = set(), set()
    for L in pa.supported_lengths():
        d = pa.plan_info(L)
        if d["row_shape"] and d["row_shape"] not in seen_row:
            seen_row.add(d["row_shape"])
            lens.add(L)
        if d["col_shape"] and d["col_shape"] not in seen_col:
            seen_col.add(d["col_shape"])
            lens.add(L)
    return [(L, pa.plan_info(L)["row_shape"], pa.plan_info(L)["col_shape"]) for L in sorted(lens)]


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
    assert len({r for _, r, _ in SHAPES}) >= 15 and len({c for _, _, c in SHAPES}) >= 5
    for L, r, c in SHAPES:
        assert r or c, L


@pytest.mark.parametrize("L,sh,cs", SHAPES, ids=[f"L{L}_row{r}_col{c}" for L, r, c in SHAPES])
def test_fixed_shapes_match_oracle(L, sh, cs):
    n, m = block_for(L)
    d = pa.plan_info(L)
    print("L=%d R=%d C=%d row shape %d column shape %d: n=%d m=%d" % (L, d["rows"], d["cols"], sh, cs, n, m),
          flush=True)
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


@pytest.mark.parametrize("a,w,general", [(7, 16, "row"), (9, 32, "column"), (0, 0, "")])
def test_general_kernels_at_a_fixed_shape_length(a, w, general):
    # L = 3 * 2^19: under R = 128 its rows of 12,288 values have no fixed
    # row kernel; R = 512 with 32-column tiles has no fixed column kernel;
    # the default geometry has both
    L = 3 * 2**19
    d = pa.plan_info(L, a, w)
    assert (d["row_shape"] == 0) == (general == "row") and (d["col_shape"] == 0) == (general == "column")
    n, m = block_for(L)
    key, seed = wl.key_and_seed(71, n, m, 0)
    want = oracle.toeplitz_hash(key, n, seed, m)
    dk, ds = dev(key), dev(seed)
    try:
        pa.tune_set(L, 0, a, w)
        assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want)
        pa.tune_set(L, 1, a, w)
        outs = [torch.zeros(wl.words(m), dtype=torch.int64, device="cuda") for _ in range(2)]
        pa.toeplitz_hash_batched([(dk, n, ds, m, o) for o in outs])
        for o in outs:
            assert np.array_equal(host(o, m), want)
    finally:
        pa.tune_set(L, 0, 0, 0)
        pa.tune_set(L, 1, 0, 0)


def extreme_blocks(L, m):
    """The largest and the smallest n with transform length L for an m that
    ends inside a word: the output window then ends on L's last word, or
    the key just exceeds the next shorter length."""
    words_m = (m + 63) // 64
    n_max = L - 64 * words_m + 1
    shorter = max([x for x in pa.supported_lengths() if x < L], default=0)
    n_min = max(m, 64 * (shorter // 64 - words_m) + 2)
    out = []
    for n in (n_max, n_min):
        if n >= m and pa.transform_len(n, m) == L:
            out.append(n)
    return out


@pytest.mark.parametrize("L,sh,cs", SHAPES, ids=[f"L{L}_row{r}_col{c}" for L, r, c in SHAPES])
def test_fixed_shapes_at_the_ends_of_each_length(L, sh, cs):
    m = 1_037
    ns = extreme_blocks(L, m)
    assert ns, L
    for n in ns:
        print("L=%d n=%d m=%d" % (L, n, m), flush=True)
        key, seed = wl.key_and_seed(80 + sh, n, m, cs)
        want = oracle.toeplitz_hash(key, n, seed, m)
        dk, ds = dev(key), dev(seed)
        assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want), ("plain", n)
        outs = [torch.zeros(wl.words(m), dtype=torch.int64, device="cuda") for _ in range(2)]
        pa.toeplitz_hash_batched([(dk, n, ds, m, o) for o in outs])
        for o in outs:
            assert np.array_equal(host(o, m), want), ("batched", n)


WIDE = [(L, a, w) for L, a, w in [(393216, 7, 64), (1572864, 8, 64), (1572864, 8, 32)]]


@pytest.mark.parametrize("L,a,w", WIDE, ids=[f"L{L}_R{2**a}_W{w}" for L, a, w in WIDE])
def test_wide_tile_column_shapes_match_oracle(L, a, w):
    # column kernels compiled for 32- and 64-column tiles, which batches of
    # these lengths may be tuned to
    assert pa.plan_info(L, a, w)["col_shape"] != 0
    n, m = block_for(L)
    key, seed = wl.key_and_seed(90 + w, n, m, a)
    want = oracle.toeplitz_hash(key, n, seed, m)
    dk, ds = dev(key), dev(seed)
    try:
        for cls in (0, 1):
            pa.tune_set(L, cls, a, w)
        assert np.array_equal(host(pa.toeplitz_hash(dk, n, ds, m), m), want)
        outs = [torch.zeros(wl.words(m), dtype=torch.int64, device="cuda") for _ in range(3)]
        pa.toeplitz_hash_batched([(dk, n, ds, m, o) for o in outs])
        for o in outs:
            assert np.array_equal(host(o, m), want)
    finally:
        for cls in (0, 1):
            pa.tune_set(L, cls, 0, 0)


@pytest.mark.parametrize("L", [393216, 1572864])
def test_many_block_forward_pass_on_wide_tiles(L):
    # a batch with at least 1024 forward tiles of 64 columns runs the
    # forward column pass on them (the plan's tiles are 16 columns wide;
    # the inverse pass keeps those)
    d = pa.plan_info(L)
    assert d["tile_width"] == 16 and pa.plan_info(L, 0, 64)["col_shape"] != 0
    count = -(-1024 // (2 * d["cols"] // 64))
    m = 20_037
    n = int(L * 0.9)
    assert pa.transform_len(n, m) == L
    blocks, want = [], []
    for i in range(count):
        key, seed = wl.key_and_seed(95, n, m, i)
        want.append(oracle.toeplitz_hash(key, n, seed, m))
        blocks.append((dev(key), n, dev(seed), m, torch.zeros(wl.words(m), dtype=torch.int64, device="cuda")))
    print("L=%d: %d blocks" % (L, count), flush=True)
    pa.toeplitz_hash_batched(blocks)
    for i, b in enumerate(blocks):
        assert np.array_equal(host(b[4], m), want[i]), i
