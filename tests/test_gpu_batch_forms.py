"""Both launch forms of a batched call against the CPU oracle (needs a GPU).

The flat form runs each pass as a few launches whose grids cover the blocks
of every length in a class (the kernels find their block by a search over
the launch's segment array); the lanes form runs each length group's own
three launches on concurrent stream lanes.  PA_BATCH_FORM selects the form
of the calls and graphs created while it is set.  Every block of an uneven
batch (many lengths, several launch classes per pass), in both forms, as a
direct call and as graph replays, must equal the oracle word for word;
the modified Toeplitz form likewise.
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


@pytest.fixture(autouse=True)
def _form_env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    old = os.environ.get("PA_BATCH_FORM")
    yield
    if old is None:
        os.environ.pop("PA_BATCH_FORM", None)
    else:
        os.environ["PA_BATCH_FORM"] = old


@pytest.fixture(scope="module")
def uneven():
    g = np.random.default_rng(61)
    items = []
    for i in range(48):
        n = int(round(2.0 ** g.uniform(12, 21)))
        m = max(1, int(round(n * g.uniform(0.05, 0.5))))
        key, seed = wl.key_and_seed(62, n, m, i)
        items.append((key, seed, n, m, oracle.toeplitz_hash(key, n, seed, m)))
    assert len({pa.transform_len(n, m) for _, _, n, m, _ in items}) >= 10
    return items


def _blocks(items):
    return [(dev(k), n, dev(s), m, torch.full((wl.words(m),), -1, dtype=torch.int64, device="cuda"))
            for k, s, n, m, _ in items]


def _check(blocks, items, what):
    torch.cuda.synchronize()
    bad = [i for i, (b, it) in enumerate(zip(blocks, items))
           if not np.array_equal(b[4].cpu().numpy().view(np.uint64)[: wl.words(it[3])], it[4])]
    assert not bad, "%s: blocks differing from the oracle: %s" % (what, bad[:10])


@pytest.mark.parametrize("form", ["flat", "lanes"])
def test_uneven_batch_in_each_form(form, uneven):
    os.environ["PA_BATCH_FORM"] = form
    blocks = _blocks(uneven)
    pa.toeplitz_hash_batched(blocks)
    _check(blocks, uneven, form + " direct call")
    # reversed submission order: same per-block results
    rblocks = _blocks(uneven[::-1])
    pa.toeplitz_hash_batched(rblocks)
    _check(rblocks, uneven[::-1], form + " reversed")


@pytest.mark.parametrize("form", ["flat", "lanes"])
def test_graph_in_each_form(form, uneven):
    os.environ["PA_BATCH_FORM"] = form
    blocks = _blocks(uneven)
    with pa.BatchGraph(blocks) as g:
        for rep in range(3):
            g.launch()
            _check(blocks, uneven, "%s graph replay %d" % (form, rep))
            for b in blocks:
                b[4].fill_(-1)
            torch.cuda.synchronize()


@pytest.mark.parametrize("form", ["flat", "lanes"])
def test_modified_batch_in_each_form(form):
    os.environ["PA_BATCH_FORM"] = form
    g = np.random.default_rng(63)
    items, blocks = [], []
    for i in range(20):
        n = int(round(2.0 ** g.uniform(12, 20)))
        m = max(1, min(n - 1, int(round(n * g.uniform(0.05, 0.5)))))
        key = wl.random_bits(n, wl.rng(64, wl.ROLE_KEY, i))
        v = wl.random_bits(n - 1, wl.rng(64, wl.ROLE_SEED, i))
        items.append((key, v, n, m, oracle.modified_toeplitz_hash(key, n, v, m)))
        blocks.append((dev(key), n, dev(v), m, torch.full((wl.words(m),), -1, dtype=torch.int64, device="cuda")))
    pa.modified_toeplitz_hash_batched(blocks)
    _check(blocks, items, form + " modified")


def _set_other_geometries(lengths, rng):
    """A valid non-default batch-class geometry for every length (other row
    count, wider tiles, another first row round, a fixed row workgroup)."""
    chosen = {}
    for L in lengths:
        a0 = int(pa.plan_info(L)["rows"]).bit_length() - 1
        cands = [(a, w, rf, rt) for a in (a0 - 1, a0 + 1, a0) for w in (64, 32, 16) for rf in (0, 2, 3, 4)
                 for rt in (512, 768, 1024, 0)]
        rng.shuffle(cands)
        for a, w, rf, rt in cands:
            if (a, w, rf, rt) == (a0, 16, 0, 0):
                continue
            try:
                pa.tune_set(L, 1, a, w, row_first=rf, row_threads=rt)
            except pa.PAError:
                continue
            chosen[L] = (a, w, rf, rt)
            break
    return chosen


@pytest.mark.parametrize("form", ["flat", "lanes"])
def test_uneven_batch_with_tuned_geometries(form, uneven):
    # the batch kernels with geometries an autotune may pick (each length
    # its own), direct and replayed, against the oracle
    os.environ["PA_BATCH_FORM"] = form
    lengths = sorted({pa.transform_len(n, m) for _, _, n, m, _ in uneven})
    chosen = _set_other_geometries(lengths, np.random.default_rng(65 if form == "flat" else 66))
    try:
        assert len(chosen) == len(lengths)
        blocks = _blocks(uneven)
        pa.toeplitz_hash_batched(blocks)
        _check(blocks, uneven, form + " tuned geometries %s" % chosen)
        for b in blocks:
            b[4].fill_(-1)
        with pa.BatchGraph(blocks) as g:
            g.launch()
            _check(blocks, uneven, form + " tuned geometries, graph")
    finally:
        for L in lengths:
            pa.tune_set(L, 1, 0, 0)
