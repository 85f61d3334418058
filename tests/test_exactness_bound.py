"""Host checks of the exactness precondition of the transform arithmetic.

The kernels compute a*w mod P (P = 27*2^20 + 1) with three fp64 FMAs:
t = fma(a, w/P, M), qP = fma(t, P, -M*P), r = fma(a, w, -qP), M = 1.5*2^52.
This is exact, with |r| <= P/2 + 4, when |a| <= 22 P and |w| <= P/2 + 4
(the twiddles are symmetric representatives, |w| <= P/2; a seed spectrum
value is a reduced residue, |w| <= P/2 + 4).  Butterflies add unreduced
values, so magnitudes grow stage by stage between multiplications.

1. The three-FMA product and the canonical reduction are checked on a
   model with exactly rounded FMAs (Python fractions), at the extremes of
   the stated ranges and on random operands.
2. For every supported transform length and every four-step split that the
   library accepts, the worst-case magnitude reaching every modular
   product, every int32 store and the final canonical reduction is derived
   from the plan's round structure (pa_plan_describe) and checked against
   22 P and 2^31.
"""
from fractions import Fraction

import numpy as np
import pytest

import paper_1809_07592_amd as pa

P = 27 * 2**20 + 1
MAGIC = 1.5 * 2.0**52
NEG_MAGIC_P = -(MAGIC * P)
PINV = 1.0 / P
LIMIT = 22 * P           # largest |a| the product accepts
B_MUL = P // 2 + 4       # largest |result| of a product (and of a symmetric reduction)


def fma(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def mulmod(a: float, w: float) -> float:
    wp = w / P
    t = fma(a, wp, MAGIC)
    qp = fma(t, float(P), NEG_MAGIC_P)
    return fma(a, w, -qp)


def canonical(a: float) -> float:
    t = fma(a, PINV, MAGIC)
    qp = fma(t, float(P), NEG_MAGIC_P)
    r = a - qp
    return r + P if r < 0 else r


def test_constants_are_exact_doubles():
    assert float(int(NEG_MAGIC_P)) == NEG_MAGIC_P and int(NEG_MAGIC_P) == -3 * 2**51 * P
    assert LIMIT * (P // 2 + 4) < 2**53       # a*w and q*P are exact in a double


@pytest.mark.parametrize("seed", range(4))
def test_three_fma_product_is_exact_on_its_range(seed):
    g = np.random.default_rng(seed)
    edges = [0, 1, -1, P // 2, -(P // 2), P, -P, LIMIT, -LIMIT, LIMIT - 1, 12345 * 1789]
    ws = [0, 1, -1, P // 2, -(P // 2), P // 2 + 4, -(P // 2 + 4), 3, 28311]
    cases = [(a, w) for a in edges for w in ws]
    cases += [(int(a), int(w)) for a, w in zip(g.integers(-LIMIT, LIMIT + 1, 400), g.integers(-(P // 2), P // 2 + 1, 400))]
    for a, w in cases:
        r = mulmod(float(a), float(w))
        assert r == int(r), (a, w)
        assert (int(r) - a * w) % P == 0, (a, w, r)
        assert abs(r) <= B_MUL, (a, w, r)


def test_canonical_reduction_on_its_range():
    g = np.random.default_rng(9)
    vals = [0, 1, -1, P - 1, P, P + 1, -P, LIMIT, -LIMIT, 7 * P + 3] + [int(v) for v in g.integers(-LIMIT, LIMIT + 1, 500)]
    for a in vals:
        r = canonical(float(a))
        assert 0 <= r < P and (int(r) - a) % P == 0, (a, r)


def supported_lengths():
    out = []
    for k in range(7, 21):
        for j in range(4):
            L = 2**k * 3**j
            if 4096 <= L <= 27 * 2**20:
                out.append(L)
    return sorted(out)


def stage_radices(round_sizes):
    """Radix of every elementary stage of a transform, from its round sizes
    (each round holds 3^a 2^b values: a radix-3 and b radix-2 stages)."""
    rad = []
    for r in round_sizes:
        while r % 3 == 0:
            rad.append(3)
            r //= 3
        while r % 2 == 0:
            rad.append(2)
            r //= 2
        assert r == 1
    return rad


def run_stages(bound, radices, checks, what, first_trivial=False):
    """Worst-case magnitude through butterfly stages: a radix-2 stage adds
    one product (P/2 + 4) to the unmultiplied input, a radix-3 stage two;
    every multiplied input must lie within the product's range.  A first
    stage whose factors are all 1 adds its inputs unmultiplied instead."""
    for i, r in enumerate(radices):
        if i == 0 and first_trivial:
            bound += (r - 1) * bound
            continue
        checks.append((what, bound))
        bound += (r - 1) * B_MUL
    return bound


def splits(L):
    seen = []
    for a in range(1, 11):
        for w in (0, 16, 32, 64):
            try:
                info = pa.plan_info(L, a, w)
            except pa.PAError:
                continue
            key = (info["rows"], tuple(info["col_round_size"]), tuple(info["row_round_size"]))
            if key not in seen:
                seen.append(key)
                yield info


def test_every_plan_stays_within_the_exact_range():
    worst = 0
    nplans = 0
    for L in supported_lengths():
        for info in splits(L):
            nplans += 1
            col = stage_radices(info["col_round_size"])
            row = stage_radices(info["row_round_size"])
            assert np.prod(col) == info["rows"] and np.prod(row) == info["cols"]
            checks, stores = [], []
            # P1: bits (|v| <= 1) through the forward column stages (the
            # first unmultiplied), the four-step twist (a product), int32 store
            b = run_stages(1, col, checks, "P1 stage", first_trivial=True)
            checks.append(("P1 twist", b))
            stores.append(B_MUL)
            # P2: forward row stages (first unmultiplied) on reduced inputs,
            # reduction of the seed spectrum and the pointwise product,
            # inverse row stages (the first unmultiplied), unreduced int32 store
            b = run_stages(B_MUL, row, checks, "P2 forward stage", first_trivial=True)
            checks.append(("P2 spectrum reduction / pointwise product", b))
            b = run_stages(B_MUL, row[::-1], checks, "P2 inverse stage", first_trivial=True)
            stores.append(b)
            # P3: inverse twist (a product), inverse column stages (the first
            # unmultiplied), then the canonical residue
            checks.append(("P3 twist", b))
            b = run_stages(B_MUL, col[::-1], checks, "P3 stage", first_trivial=True)
            checks.append(("P3 canonical", b))
            for what, v in checks:
                assert v <= LIMIT, (L, info["rows"], what, v / P)
                worst = max(worst, v)
            assert max(stores) < 2**31
    assert nplans >= len(supported_lengths())
    # the largest magnitude any plan reaches, in units of P (about 9 P)
    assert worst <= 10 * P
