"""Host-only checks of the C ABI (no GPU needed).

The library must load, export every function include/pa.h declares, and
reject bad arguments synchronously before any HIP call.  Length selection
is checked against an independent computation of the smallest 2^k 3^j.
"""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1809_07592_amd as pa
from paper_1809_07592_amd import build as pa_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pa.LIB_PATH):
        pa_build.build()
    return pa.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "pa_toeplitz_hash" in names and "pa_toeplitz_hash_batched" in names
    out = subprocess.run(["nm", "-D", "--defined-only", pa.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pa_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


FAKE = 0x10000  # non-null, never dereferenced: validation fails first


@pytest.mark.parametrize("key,n,seed,m,out,status", [
    (None, 10, FAKE, 5, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, None, 5, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 5, None, pa.PA_ERR_INVALID_ARG),
    (FAKE, 0, FAKE, 1, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 0, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 11, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 30_000_000, FAKE, 1, FAKE, pa.PA_ERR_UNSUPPORTED_SIZE),
    (FAKE, 20_000_000, FAKE, 9_000_000, FAKE, pa.PA_ERR_UNSUPPORTED_SIZE),
])
def test_rejects_before_device_work(lib, key, n, seed, m, out, status):
    assert lib.pa_toeplitz_hash(key, n, seed, m, out, None) == status
    assert len(pa.last_error()) > 0
    assert lib.pa_toeplitz_hash_noalloc(key, n, seed, m, out, None) == status
    assert len(pa.last_error()) > 0


def test_noalloc_rejects_blocks_beyond_its_scratch(lib):
    # 8 L bytes must fit the static scratch: L <= 27 * 2^19; the next
    # supported length (27 * 2^20) is refused on the host, before any device call
    assert pa.NOALLOC_SCRATCH_BYTES == 8 * 27 * 2**19
    assert pa.transform_len(12_800_000, 1_280_000) == 27 * 2**19
    n, m = 16_000_000, 1_000_000
    L = pa.transform_len(n, m)
    assert L == 27 * 2**20
    assert lib.pa_toeplitz_hash_noalloc(FAKE, n, FAKE, m, FAKE, None) == pa.PA_ERR_UNSUPPORTED_SIZE
    assert "scratch" in pa.last_error()


def test_batched_validation(lib):
    blocks = (pa._Block * 2)()
    blocks[0] = pa._Block(FAKE, 100, FAKE, 10, FAKE)
    blocks[1] = pa._Block(FAKE, 100, FAKE, 101, FAKE)
    assert lib.pa_toeplitz_hash_batched(blocks, 2, None) == pa.PA_ERR_INVALID_ARG
    assert "block 1" in pa.last_error()
    assert lib.pa_toeplitz_hash_batched(blocks, 0, None) == pa.PA_OK
    assert lib.pa_toeplitz_hash_batched(None, 3, None) == pa.PA_ERR_INVALID_ARG


@pytest.mark.parametrize("key,n,v,m,out,status", [
    (FAKE, 100, FAKE, 100, FAKE, pa.PA_ERR_INVALID_ARG),   # m = n: V would have no column
    (FAKE, 100, FAKE, 0, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 1, FAKE, 1, FAKE, pa.PA_ERR_INVALID_ARG),
    (None, 100, FAKE, 10, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 100, None, 10, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 100, FAKE, 10, None, pa.PA_ERR_INVALID_ARG),
    (FAKE, 40_000_000, FAKE, 10, FAKE, pa.PA_ERR_UNSUPPORTED_SIZE),
])
def test_modified_rejects_before_device_work(lib, key, n, v, m, out, status):
    assert lib.pa_modified_toeplitz_hash(key, n, v, m, out, None) == status
    blocks = (pa._Block * 1)()
    blocks[0] = pa._Block(key, n, v, m, out)
    assert lib.pa_modified_toeplitz_hash_batched(blocks, 1, None) == status
    assert "block 0" in pa.last_error()


def test_graph_validation(lib):
    h = ctypes.c_void_p()
    blocks = (pa._Block * 2)()
    blocks[0] = pa._Block(FAKE, 100, FAKE, 10, FAKE)
    blocks[1] = pa._Block(FAKE, 100, FAKE, 101, FAKE)
    assert lib.pa_graph_create(blocks, 2, 0, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert "block 1" in pa.last_error() and not h.value
    assert lib.pa_graph_create(blocks, 0, 0, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_graph_create(None, 2, 0, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_graph_create(blocks, 1, 0, None) == pa.PA_ERR_INVALID_ARG
    blocks[1] = pa._Block(FAKE, 100, FAKE, 100, FAKE)   # m = n: invalid only for the modified form
    assert lib.pa_graph_create(blocks, 2, 1, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_graph_launch(None, None) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_graph_destroy(None) == pa.PA_OK
    assert lib.pa_graph_block_count(None) == 0


def test_fft_pair_validation(lib):
    err, fb = ctypes.c_double(), ctypes.c_int()
    F2 = FAKE + 4096
    call = lambda *a: lib.pa_toeplitz_hash_pair_fft(*a, None, ctypes.byref(err), ctypes.byref(fb))
    assert call(FAKE, F2, 100, FAKE, 10, FAKE, FAKE, 0.25) == pa.PA_ERR_INVALID_ARG      # outputs overlap
    assert call(FAKE, None, 100, FAKE, 10, FAKE, F2, 0.25) == pa.PA_ERR_INVALID_ARG
    assert call(FAKE, F2, 100, FAKE, 101, FAKE, F2 + 64, 0.25) == pa.PA_ERR_INVALID_ARG  # m > n
    assert call(FAKE, F2, 100, FAKE, 10, FAKE, F2 + 64, 0.75) == pa.PA_ERR_INVALID_ARG   # guard > 1/2
    assert call(FAKE, F2, 100, FAKE, 10, FAKE, F2 + 64, -1.0) == pa.PA_ERR_INVALID_ARG
    assert call(FAKE, F2, 16_000_000, FAKE, 2_000_000, FAKE, F2 + 64, 0.25) == pa.PA_ERR_UNSUPPORTED_SIZE


def test_fft_pair_lengths(lib):
    # power of two covering the convolution window, at least 2^12, at most 2^24
    assert pa.fft_pair_transform_len(1, 1) == 4096
    assert pa.fft_pair_transform_len(1_000_000, 250_000) == 2**21
    assert pa.fft_pair_transform_len(12_800_000, 1_280_000) == 2**24
    assert pa.fft_pair_transform_len(16_000_000, 2_000_000) == 0
    assert pa.fft_pair_transform_len(10, 11) == 0


def test_final_key_length_follows_eq1():
    # r = n - t - s (Eq. 1: s = n - t - r), clamped at 0
    assert pa.final_key_length(1_000_000, 200_000, 100) == 799_900
    assert pa.final_key_length(100, 40, 60) == 0
    assert pa.final_key_length(100, 101, 0) == 0
    assert pa.final_key_length(100, 0, 2**63) == 0
    assert pa.final_key_length(2**62, 1, 1) == 2**62 - 2


def test_plan_validation(lib):
    h = ctypes.c_void_p()
    assert lib.pa_plan_create(None, 100, 0, None, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_plan_create(FAKE, 0, 0, None, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_plan_create(FAKE, 100, 5000, None, ctypes.byref(h)) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_plan_create(FAKE, 40_000_000, 0, None, ctypes.byref(h)) == pa.PA_ERR_UNSUPPORTED_SIZE
    assert lib.pa_plan_hash(None, FAKE, 10, 5, FAKE, None) == pa.PA_ERR_INVALID_ARG
    assert lib.pa_plan_destroy(None) == pa.PA_OK
    assert lib.pa_plan_transform_len(None) == 0


def smallest_len(req):
    best = None
    for k in range(7, 21):
        for j in range(4):
            L = 2**k * 3**j
            if 4096 <= L <= 27 * 2**20 and L >= req and (best is None or L < best):
                best = L
    return best or 0


@pytest.mark.parametrize("n,m", [(1, 1), (64, 64), (65, 1), (262_144, 65_536), (1_000_000, 250_000),
                                 (12_800_000, 1_280_000), (4096, 4096), (24_000_000, 4_300_000)])
def test_transform_length_choice(lib, n, m):
    req = 64 * ((n - 1 + 63) // 64 + (m + 63) // 64)
    assert pa.transform_len(n, m) == smallest_len(req)
    assert pa.workspace_bytes(n, m) == 8 * smallest_len(req)


def test_paper_config_lengths(lib):
    # mixed-radix lengths cut the padding of the power-of-two choice
    assert pa.transform_len(1_000_000, 250_000) == 3 * 2**19
    assert pa.transform_len(12_800_000, 1_280_000) == 27 * 2**19
    assert pa.transform_len(262_144, 65_536) == 3 * 2**17


def test_status_strings(lib):
    for code, name in [(0, "PA_OK"), (1, "PA_ERR_INVALID_ARG"), (2, "PA_ERR_UNSUPPORTED_SIZE"),
                       (3, "PA_ERR_OUT_OF_MEMORY"), (4, "PA_ERR_DEVICE"), (5, "PA_ERR_BUSY")]:
        assert pa.status_string(code) == name
    assert "gfx950" in pa.version()


def test_modulus_facts():
    # P = 27*2^20 + 1 is prime with primitive root 5; P > every supported length
    from sympy import isprime, n_order
    P = 27 * 2**20 + 1
    assert isprime(P) and n_order(5, P) == P - 1
    assert P > pa.MAX_TRANSFORM_LEN
    # 3-FMA product exactness needs |a w| < 2^53 for |a| <= 22 P, |w| <= P/2
    assert 22 * P * (P // 2) < 2**53


def test_product_never_touches_oracle():
    pkg = os.path.join(ROOT, "paper_1809_07592_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "toeplitz_oracle" not in text and "liboracle" not in text, f


def _check_geometry(d, L):
    R, C, W = d["rows"], d["cols"], d["tile_width"]
    assert R * C == L and C % 64 == 0 and W in (16, 32, 64) and C % W == 0
    assert 1 <= d["col_threads"] <= 512 and d["col_threads"] % 64 == 0
    assert 1 <= d["row_threads"] <= 1024 and d["row_threads"] % 64 == 0
    assert d["col_lds_bytes"] <= 160 * 1024 and d["row_lds_bytes"] <= 160 * 1024
    prod = 1
    for r in d["col_round_size"]:
        assert r in (2, 4, 8, 16)
        prod *= r
    assert prod == R
    prod = 1
    rr = d["row_round_size"]
    for i, r in enumerate(rr):
        # rows: a first round of at most 12 values that takes the radix-3
        # stages, except that 27 | C splits as 9 then 3 or 6; then radix-2
        # rounds of at most 8
        if i == 0:
            assert r <= 12
        elif i == 1 and rr[0] == 9 and C % 27 == 0:
            assert r in (3, 6)
        else:
            assert r in (2, 4, 8)
        prod *= r
    assert prod == C and d["row_rounds"] >= 2
    # the output-packing ballots need the first column round to cover
    # whole 64-lane waves
    assert (R // d["col_round_size"][0]) * W % 64 == 0


def test_every_supported_length_has_a_valid_launch_geometry(lib):
    for L in pa.supported_lengths():
        _check_geometry(pa.plan_info(L), L)


def test_every_accepted_split_is_a_valid_launch_geometry(lib):
    """Every (R, W) the planner accepts (what tuning may select) satisfies
    the kernels' launch assumptions, and each length has several."""
    for L in pa.supported_lengths():
        accepted = 0
        for a in range(1, 11):
            for w in (16, 32, 64):
                try:
                    d = pa.plan_info(L, a, w)
                except pa.PAError:
                    continue
                assert d["rows"] == 2**a and d["tile_width"] == w
                _check_geometry(d, L)
                accepted += 1
        assert accepted >= 1, L


def test_default_geometries_run_fixed_row_kernels(lib):
    """Every length from 2^16 up runs, in its default geometry, row and
    column kernels compiled for its transforms' shapes; one shape per
    length and round split (and, for columns, tile width); a geometry no
    fixed kernel covers runs the general kernels."""
    shape_of, col_shape_of = {}, {}
    for L in pa.supported_lengths():
        d = pa.plan_info(L)
        if L >= 2**16:
            assert d["row_shape"] != 0, (L, d["cols"], d["row_round_size"])
            assert d["col_shape"] != 0, (L, d["rows"], d["col_round_size"])
        if d["row_shape"]:
            key = (d["cols"], tuple(d["row_round_size"]))
            assert shape_of.setdefault(key, d["row_shape"]) == d["row_shape"], key
        if d["col_shape"]:
            key = (d["rows"], tuple(d["col_round_size"]), d["tile_width"])
            assert col_shape_of.setdefault(key, d["col_shape"]) == d["col_shape"], key
    assert len(set(shape_of.values())) == len(shape_of) >= 15
    assert len(set(col_shape_of.values())) == len(col_shape_of) >= 5
    # R = 512 with 32-column tiles: the general column kernels; R = 256
    # with 64-column tiles (a batch tuning choice): a fixed one
    assert pa.plan_info(3 * 2**19, log2_rows=9, tile_width=32)["col_shape"] == 0
    assert pa.plan_info(3 * 2**19, log2_rows=8, tile_width=64)["col_shape"] != 0
    # R = 128 gives rows of 12288 values: no fixed kernel
    assert pa.plan_info(3 * 2**19, log2_rows=7)["row_shape"] == 0
    # the same row transform inside another length uses the same kernel
    assert pa.plan_info(3 * 2**18, log2_rows=7)["row_shape"] == pa.plan_info(3 * 2**19)["row_shape"]


def test_geometry_overrides(lib):
    d = pa.plan_info(3 * 2**19, log2_rows=9, tile_width=32)
    assert (d["rows"], d["cols"], d["tile_width"]) == (512, 3072, 32)
    with pytest.raises(pa.PAError):
        pa.plan_info(3 * 2**19, log2_rows=16)
    with pytest.raises(pa.PAError):
        pa.plan_info(12345)


@pytest.mark.parametrize("a,na,b,nb,L,out,status", [
    (None, 10, FAKE, 10, 4096, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, None, 10, 4096, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 10, 4096, None, pa.PA_ERR_INVALID_ARG),
    (FAKE, 0, FAKE, 10, 4096, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 4097, FAKE, 10, 4096, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 4097, 4096, FAKE, pa.PA_ERR_INVALID_ARG),
    (FAKE, 10, FAKE, 10, 5000, FAKE, pa.PA_ERR_UNSUPPORTED_SIZE),
])
def test_cyclic_convolution_rejects_before_device_work(lib, a, na, b, nb, L, out, status):
    assert lib.pa_cyclic_convolution(a, na, b, nb, L, out, None) == status
    assert len(pa.last_error()) > 0


def test_plan_spectrum_rejects_null(lib):
    assert lib.pa_plan_spectrum(None, FAKE, None) == pa.PA_ERR_INVALID_ARG
