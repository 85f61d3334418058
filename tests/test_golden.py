"""Stored cases of tests/golden/toeplitz_cases.txt (written by
make_golden.py from the CPU oracle).  On the CPU each stored output is
checked against the definition written out with the explicit matrix and
against the oracle as it now stands; on the GPU the HIP path must
reproduce it bit for bit."""
import os

import numpy as np
import pytest

import oracle
import paper_1809_07592_amd as pa
from paper_1809_07592_amd import workloads as wl

CASES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "toeplitz_cases.txt")


def load_cases():
    out = []
    with open(CASES) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, n, m, key, seed, y = line.split()
            out.append((kind, int(n), int(m), int(key, 16), int(seed, 16), int(y, 16)))
    return out


def words_of(v: int, nbits: int) -> np.ndarray:
    nw = wl.words(nbits)
    return np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(nw)], dtype=np.uint64)


def bit(v: int, k: int) -> int:
    return (v >> k) & 1


def plain_by_matrix(n, m, x, s):
    """y_i = XOR_j T[i][j] x_j with T[i][j] = s[i - j + n - 1] (Sec. 2.2)."""
    y = 0
    for i in range(m):
        acc = 0
        for j in range(n):
            acc ^= bit(s, i - j + n - 1) & bit(x, j)
        y |= acc << i
    return y


def modified_by_matrix(n, m, x, v):
    """y = x[0:m] XOR V x[m:n], V[i][j] = v[i - j + (n - m) - 1] (Eq. 2-3)."""
    k = n - m
    y = 0
    for i in range(m):
        acc = bit(x, i)
        for j in range(k):
            acc ^= bit(v, i - j + k - 1) & bit(x, m + j)
        y |= acc << i
    return y


def test_cases_file_is_complete():
    cases = load_cases()
    kinds = {c[0] for c in cases}
    assert kinds == {"plain", "modified"} and len(cases) >= 10


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: "%s-%d-%d" % c[:3])
def test_stored_output_matches_definition_and_oracle(case):
    kind, n, m, x, s, y = case
    if n * m <= 600_000:  # explicit matrix: small cases only
        ref = plain_by_matrix(n, m, x, s) if kind == "plain" else modified_by_matrix(n, m, x, s)
        assert ref == y
    key = words_of(x, n)
    if kind == "plain":
        got = oracle.toeplitz_hash(key, n, words_of(s, n + m - 1), m)
    else:
        got = oracle.modified_toeplitz_hash(key, n, words_of(s, n - 1), m)
    assert np.array_equal(np.asarray(got, dtype=np.uint64)[: wl.words(m)], words_of(y, m))


@pytest.mark.gpu
@pytest.mark.parametrize("case", load_cases(), ids=lambda c: "%s-%d-%d" % c[:3])
def test_hip_path_reproduces_stored_output(case):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kind, n, m, x, s, y = case
    dev = lambda a: torch.from_numpy(a.view(np.int64)).cuda()
    key = dev(words_of(x, n))
    if kind == "plain":
        out = pa.toeplitz_hash(key, n, dev(words_of(s, n + m - 1)), m)
    else:
        out = pa.modified_toeplitz_hash(key, n, dev(words_of(s, n - 1)), m)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64)[: wl.words(m)], words_of(y, m))
