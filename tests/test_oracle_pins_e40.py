"""Pins of the oracle's modulus-3^40 generator (the longer-period variant
that Section 2 names) against the mathematics: the order of 2 modulo 3^40,
the floor(3^e/2) identity behind Eq. 2 up to e = 40, the truncated alpha_{2,3}
sum (itself pinned against the exact expansion of alpha at small e), Python's
big-integer pow and exact rational rounding."""
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc

M = 3 ** 40
P = 2 * 3 ** 39


def test_e40_constants_and_period():
    assert orc.E40_MOD == M and M < 2 ** 64 and 2 ** 63 < M
    assert 2 ** 53 < M  # the step multiplier is 2^53 itself
    # the order of 2 is 2*3^39: 2^P = 1 and no maximal proper divisor works
    assert pow(2, P, M) == 1
    assert pow(2, P // 2, M) != 1 and pow(2, P // 3, M) != 1
    # 53 is prime to the period, so 2^53 has the same order
    assert P % 53 != 0
    assert orc.e40_skip(1, P) == 1 and orc.e40_skip(1, P // 2) != 1
    assert orc.e40_skip(1, P // 3) != 1


def test_floor_half_identity_up_to_40():
    """sum_{k=1}^{e} 3^(e-k) 2^(3^e-3^k) == floor(3^e/2) (mod 3^e) for
    e = 34..40, so Eq. 2 carries over to the larger modulus."""
    for e in range(34, 41):
        m = 3 ** e
        acc = sum(3 ** (e - k) * pow(2, 3 ** e - 3 ** k, m) for k in range(1, e + 1)) % m
        assert acc == m // 2, e
        assert orc.g_index_state(m, e) == m // 2


def test_e40_seed_equals_alpha_digit_sum():
    """Eq. 2 at modulus 3^40 equals the truncated alpha sum at the same
    position, and so do the generated states at positions a + 53 k."""
    rng = random.Random(40)
    seeds = [orc.E40_INDEX_MIN, orc.E40_INDEX_MAX, 14_000_000_000_000_000_001]
    seeds += [rng.randint(orc.E40_INDEX_MIN, orc.E40_INDEX_MAX) for _ in range(8)]
    for a in seeds:
        z0 = orc.e40_seed(a)
        assert z0 == orc.g_digit_sum(a, 40), a
        if a > orc.E40_INDEX_MAX - 53 * 600:
            continue
        zs, zn = orc.e40_gen(z0, 600, "u64")
        for k in (1, 2, 3, 17, 599, 600):
            assert int(zs[k - 1]) == orc.g_digit_sum(a + 53 * k, 40), (a, k)
        assert zn == int(zs[-1])


def test_e40_digit_sum_no_overflow():
    """Residue sums pass 2^64 at this modulus: compare with Python integers
    on positions where the partial sums are large."""
    rng = random.Random(41)
    for _ in range(30):
        n = rng.randint(M, 2 ** 64 - 1)
        want = sum(3 ** (40 - k) * pow(2, n - 3 ** k, 3 ** k) for k in range(1, 41)) % M
        assert orc.g_digit_sum(n, 40) == want


def test_e40_step_skip_and_pow():
    rng = random.Random(42)
    mult = 2 ** 53
    for _ in range(200):
        z = rng.randrange(1, M)
        if z % 3 == 0:
            continue
        assert orc.e40_step(z) == mult * z % M
        k = rng.randrange(0, 2 ** 64)
        assert orc.e40_skip(z, k) == z * pow(mult, k, M) % M
    z = orc.e40_seed(orc.E40_INDEX_MIN)
    zs, zn = orc.e40_gen(z, 5000, "u64")
    assert zn == orc.e40_skip(z, 5000)
    w = z
    for k in range(5000):
        w = w * mult % M
        if k in (0, 1, 777, 4999):
            assert int(zs[k]) == w


def test_e40_f64_rounding():
    """RN(RN(z) * RN(1/3^40)) in (0,1): Python's int-to-float conversion and
    float product are the IEEE roundings."""
    r = Fraction(float(Fraction(1, M)))
    assert float(r) == 1.0 / M
    rng = random.Random(43)
    zs = [1, 2, M - 1, M - 2, M // 2, M // 2 + 1, 2 ** 63, 2 ** 63 + 1, 2 ** 53 + 1]
    zs += [rng.randrange(1, M) for _ in range(20000)]
    zs = [z for z in zs if z % 3]
    for z in zs:
        got = orc.e40_to_f64(z)
        want = float(Fraction(float(z)) * r)
        assert got == want, z
        assert 0.0 < got < 1.0
        assert abs(Fraction(got) - Fraction(z, M)) <= Fraction(z, M) / 2 ** 51
    u, zu = orc.e40_gen(orc.e40_seed(orc.E40_INDEX_MIN), 2048, "u64")
    f, zf = orc.e40_gen(orc.e40_seed(orc.E40_INDEX_MIN), 2048, "f64")
    assert zu == zf and all(orc.e40_to_f64(int(x)) == y for x, y in zip(u, f))


def test_e40_seed_range():
    for bad in (0, M, orc.E40_INDEX_MIN - 1, 2 ** 53):
        with pytest.raises(ValueError):
            orc.e40_seed(bad)
    rng = random.Random(44)
    idx = {rng.randint(orc.E40_INDEX_MIN, orc.E40_INDEX_MAX) for _ in range(2000)}
    states = {orc.e40_seed(a) for a in idx}
    assert len(states) == len(idx)
    assert all(s % 3 and 0 < s < M for s in states)
