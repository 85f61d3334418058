"""Host-only checks of the geometry tuning table (no device work).

The split R x C of the four-step transform (Sec. 3.1, Alg. 1) is a free
choice: these tests cover the table's validation, lookup and persistence;
the GPU tests check that every split gives the same bits.
"""
import os

import pytest

import paper_1809_07592_amd as pa

L = 3 * 2**19


@pytest.fixture(autouse=True)
def _restore_defaults():
    yield
    for cls in (0, 1):
        pa.tune_set(L, cls, 0, 0)
        pa.tune_set(2**20, cls, 0, 0)


def test_default_matches_plan_describe():
    info = pa.plan_info(L)
    a, w = pa.tune_get(L, 0)
    assert (1 << a) == info["rows"] and w == info["tile_width"]
    assert pa.tune_get(L, 1) == (a, w)


def test_set_and_restore_per_class():
    a0, w0 = pa.tune_get(L, 0)
    alt = 10 if a0 != 10 else 9
    pa.tune_set(L, 1, alt, 0)
    a1, w1 = pa.tune_get(L, 1)
    assert a1 == alt
    assert pa.tune_get(L, 0) == (a0, w0)       # other class untouched
    info = pa.plan_info(L, alt, 0)
    assert w1 == info["tile_width"]
    pa.tune_set(L, 1, 0, 0)
    assert pa.tune_get(L, 1) == (a0, w0)


@pytest.mark.parametrize("args,status", [
    ((L, 2, 8, 32), pa.PA_ERR_INVALID_ARG),          # no such class
    ((L, 0, 11, 32), pa.PA_ERR_INVALID_ARG),         # more rows than allowed
    ((L, 0, 8, 48), pa.PA_ERR_INVALID_ARG),          # tile width not 16/32/64
    ((5 * 2**18, 0, 8, 32), pa.PA_ERR_UNSUPPORTED_SIZE),  # 5 does not divide p - 1
])
def test_invalid_settings_rejected(args, status):
    with pytest.raises(pa.PAError) as ei:
        pa.tune_set(*args)
    assert ei.value.status == status
    assert pa.tune_get(L, 0) == pa.tune_get(L, 1)


def test_save_load_round_trip(tmp_path):
    pa.tune_set(L, 0, 9, 32)
    pa.tune_set(2**20, 1, 7, 64)
    path = str(tmp_path / "tune.txt")
    pa.tune_save(path)
    text = open(path).read()
    assert "%d 0 9 32" % L in text and "%d 1 7 64" % 2**20 in text
    pa.tune_set(L, 0, 0, 0)
    pa.tune_set(2**20, 1, 0, 0)
    pa.tune_load(path)
    assert pa.tune_get(L, 0) == (9, 32)
    assert pa.tune_get(2**20, 1) == (7, 64)


def test_load_rejects_bad_file_atomically(tmp_path):
    path = str(tmp_path / "bad.txt")
    with open(path, "w") as f:
        f.write("# comment\n%d 0 9 32\n%d 0 99 32\n" % (L, 2**20))
    before = pa.tune_get(L, 0)
    with pytest.raises(pa.PAError) as ei:
        pa.tune_load(path)
    assert ei.value.status == pa.PA_ERR_INVALID_ARG
    assert ":3:" in str(ei.value)
    assert pa.tune_get(L, 0) == before           # nothing installed
    with open(path, "w") as f:
        f.write("%d 0 9\n" % L)
    with pytest.raises(pa.PAError):
        pa.tune_load(path)
    with pytest.raises(pa.PAError):
        pa.tune_load(os.path.join(str(tmp_path), "missing.txt"))


def test_full_geometry_set_get_and_validation():
    # 6144-column rows (L = 3 * 2^19, R = 256): the first round can take 0, 1
    # or 2 radix-2 stages after its radix-3 stage (3, 6 or 12 values)
    pa.tune_set(L, 0, 8, 16, row_first=2, row_threads=1024)
    g = pa.tune_get_geometry(L, 0)
    assert g == {"log2_rows": 8, "tile_width": 16, "row_first": 2, "row_threads": 1024}
    info = pa.plan_info(L, 8, 16)
    assert info["row_round_size"][0] == 12       # the default first round
    for bad in (dict(row_first=4), dict(row_threads=300), dict(row_threads=2048)):
        with pytest.raises(pa.PAError) as ei:
            pa.tune_set(L, 0, 8, 16, **bad)
        assert ei.value.status == pa.PA_ERR_INVALID_ARG
    assert pa.tune_get_geometry(L, 0)["row_threads"] == 1024    # unchanged by the failures
    pa.tune_set(L, 0, 0, 0)
    assert pa.tune_get_geometry(L, 0)["row_first"] == 0


def test_save_load_keeps_full_geometry_and_filters_by_architecture(tmp_path):
    pa.tune_set(L, 1, 9, 32, row_first=1, row_threads=512)
    path = str(tmp_path / "tune.txt")
    pa.tune_save(path)
    lines = [ln.split() for ln in open(path) if not ln.startswith("#")]
    assert any(ln[:6] == [str(L), "1", "9", "32", "1", "512"] and len(ln) == 7 for ln in lines)
    arch = [ln for ln in lines if ln[0] == str(L)][0][6]
    pa.tune_set(L, 1, 0, 0)
    # a line for another architecture is kept in the file but not installed
    with open(path, "a") as f:
        f.write("%d 0 10 16 0 0 gfx000\n" % L)
    pa.tune_load(path)
    assert pa.tune_get_geometry(L, 1) == {"log2_rows": 9, "tile_width": 32, "row_first": 1, "row_threads": 512}
    assert pa.tune_get(L, 0) != (10, 16)
    # a bad line of this architecture fails the whole load
    with open(path, "a") as f:
        f.write("%d 0 8 16 9 0 %s\n" % (L, arch))
    pa.tune_set(L, 1, 0, 0)
    with pytest.raises(pa.PAError):
        pa.tune_load(path)
    assert pa.tune_get_geometry(L, 1)["row_first"] == 0
