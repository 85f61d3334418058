"""The transform below the hash, on the GPU (kernel-level checks).

pa_cyclic_convolution runs the hash's own passes (forward column pass of
both inputs, row pass, inverse column pass) but stores every canonical
residue: the exact length-L cyclic convolution.  It is checked against a
direct O(L^2) convolution computed here with numpy integers (the
convolution theorem of Sec. 2.3, Eq. (4), with nothing between the
transforms and the result), on lengths 2^12, 3 * 2^11, 9 * 2^9 and
27 * 2^9 (every first-round kind of the row pass).  A unit impulse makes
the forward-inverse round trip the identity (and a shifted impulse a
rotation); all-ones inputs reach the largest values.  The resident
spectrum of a plan is the length-L transform of its seed: the unit impulse
transforms to all ones, the next unit vector to every L-th root of unity
exactly once, and a random seed to the values a CPU transform gives.
"""
import numpy as np
import pytest

import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

from bitutil import pack, unpack

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

P = 27 * 2**20 + 1
LENGTHS = [2**12, 3 * 2**11, 9 * 2**9, 27 * 2**9]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def direct_cyclic(a_bits, b_bits, L):
    """c[k] = sum_j a[j] b[(k - j) mod L], by the O(L^2) definition."""
    a = np.zeros(L, dtype=np.int64)
    b = np.zeros(L, dtype=np.int64)
    a[: a_bits.size] = a_bits
    b[: b_bits.size] = b_bits
    lin = np.convolve(a, b)                     # direct method on integers
    c = lin[:L].copy()
    c[: lin.size - L] += lin[L:]
    return c


def gpu_conv(a_bits, b_bits, L):
    out = pa.cyclic_convolution(dev(pack(a_bits)), a_bits.size, dev(pack(b_bits)), b_bits.size, L)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("L", LENGTHS)
def test_convolution_theorem_against_direct_convolution(L):
    g = np.random.default_rng(L)
    for na, nb in [(L, L), (int(L * 0.7), int(L * 0.45)), (1, L), (L - 1, 3)]:
        a = g.integers(0, 2, na).astype(np.uint8)
        b = g.integers(0, 2, nb).astype(np.uint8)
        assert np.array_equal(gpu_conv(a, b, L), direct_cyclic(a, b, L)), (L, na, nb)


@pytest.mark.parametrize("L", LENGTHS)
def test_unit_impulse_round_trip_and_rotation(L):
    g = np.random.default_rng(L + 1)
    a = g.integers(0, 2, L).astype(np.uint8)
    for k in (0, 1, 63, L // 3, L - 1):
        e = np.zeros(k + 1, dtype=np.uint8)
        e[k] = 1
        got = gpu_conv(a, e, L)
        assert np.array_equal(got, np.roll(a.astype(np.int64), k)), (L, k)


@pytest.mark.parametrize("L", LENGTHS)
def test_all_ones_reach_the_largest_values(L):
    ones = np.ones(L, dtype=np.uint8)
    assert np.array_equal(gpu_conv(ones, ones, L), np.full(L, L, dtype=np.int64))
    half = np.ones(L // 2, dtype=np.uint8)
    assert np.array_equal(gpu_conv(half, ones, L), np.full(L, L // 2, dtype=np.int64))
    assert np.array_equal(gpu_conv(half, half, L), direct_cyclic(half, half, L))


@pytest.mark.parametrize("L", LENGTHS)
def test_spectrum_of_unit_vectors(L):
    for k, check in ((0, "ones"), (1, "roots")):
        bits = np.zeros(L, dtype=np.uint8)
        bits[k] = 1
        with pa.Plan(dev(pack(bits)), L, transform_len=L) as plan:
            spec = plan.spectrum()
            torch.cuda.synchronize()
            v = spec.cpu().numpy().astype(np.int64)
        assert np.all(np.abs(v) <= P // 2 + 4)
        r = np.mod(v, P)
        if check == "ones":
            assert np.all(r == 1)
        else:
            # NTT(e_1)[f] = w^f for a primitive L-th root w: every L-th root
            # of unity exactly once, whatever the order of the output
            assert np.unique(r).size == L
            assert all(pow(int(x), L, P) == 1 for x in r[:: max(1, L // 257)])
            assert all(pow(int(x), L, P) == 1 for x in r)


def cpu_ntt(x, w):
    """Length-N transform X_k = sum_i x_i w^(ik) mod P (N = 2^a 3^b), by
    recursive decimation in time: a plain model of the transform, not of
    the kernels' rounds or order."""
    N = x.size
    if N == 1:
        return x % P
    r = 2 if N % 2 == 0 else 3
    M = N // r
    parts = [cpu_ntt(x[i::r], pow(w, r, P)) for i in range(r)]
    wk = np.ones(N, dtype=np.int64)
    for k in range(1, N):
        wk[k] = wk[k - 1] * w % P
    k = np.arange(N)
    out = np.zeros(N, dtype=np.int64)
    for i in range(r):
        out = (out + parts[i][k % M] * wk[(i * k) % N]) % P
    return out


@pytest.mark.parametrize("L", LENGTHS)
def test_spectrum_values_match_a_cpu_transform(L):
    # the resident spectrum of a random seed holds the values of its
    # length-L transform (in the kernels' own order): the same multiset
    # as a CPU transform at any primitive L-th root of unity
    g = np.random.default_rng(L + 7)
    bits = g.integers(0, 2, L).astype(np.uint8)
    with pa.Plan(dev(pack(bits)), L, transform_len=L) as plan:
        spec = plan.spectrum()
        torch.cuda.synchronize()
        v = spec.cpu().numpy().astype(np.int64)
    assert np.all(np.abs(v) <= P // 2 + 4)
    w = pow(5, (P - 1) // L, P)
    want = cpu_ntt(bits.astype(np.int64), w)
    assert np.array_equal(np.sort(np.mod(v, P)), np.sort(want))


def test_bits_of_the_convolution_give_the_hash():
    # y_i is bit n-1+i of the linear convolution s * x (mod 2): the
    # residues of a cyclic convolution long enough not to wrap, read at
    # those positions, equal the hash
    n, m = 3000, 700
    key, seed = wl.key_and_seed(90, n, m, 0)
    L = 2**12
    x = unpack(key, n)
    s = unpack(seed, n + m - 1)
    c = gpu_conv(s, x, L)
    want = unpack(pa.toeplitz_hash(dev(key), n, dev(seed), m).cpu().numpy().view(np.uint64), m)
    assert np.array_equal((c[n - 1: n - 1 + m] & 1).astype(np.uint8), want)
