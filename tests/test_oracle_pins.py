"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-derives the oracle's own formula with the oracle's own
code: each compares it with something independent -- constants printed in
the paper, the binary expansion of alpha_{2,3} computed exactly from its
definition (Section 2), the order of 2 modulo 3^33, brute-force enumeration of
the small analogues, Python's own big-integer ``pow`` and exact rational
arithmetic for the rounding of the variates.
"""
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

M = 3 ** 33
P = 2 * 3 ** 32
H = M // 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            name, expr = (s.strip() for s in line.split("=", 1))
            if expr.lower().startswith("0x"):
                vals[name] = int(expr, 16)
                continue
            # products/sums/powers of integers only, e.g. "2*3^32", "3^33+100"
            assert set(expr) <= set("0123456789*+^"), expr
            total = 0
            for term in expr.split("+"):
                prod = 1
                for fac in term.split("*"):
                    if "^" in fac:
                        b, e = fac.split("^")
                        prod *= int(b) ** int(e)
                    else:
                        prod *= int(fac)
                total += prod
            vals[name] = total
    return vals


def test_printed_constants():
    g = _golden()
    assert g["modulus"] == 3 ** 33 == orc.MOD
    # The Barrett bound is garbled in print; mu is read as floor(2^(2k)/m), k=53.
    assert g["mu"] == 2 ** 106 // g["modulus"]
    assert g["mask53"] == 2 ** 53 - 1 and g["two53"] == 2 ** 53
    assert g["mask54"] == 2 ** 54 - 1 and g["two54"] == 2 ** 54
    assert g["period"] == P
    assert g["index_min"] == orc.INDEX_MIN == wl.INDEX_MIN
    assert g["index_max"] == orc.INDEX_MAX == wl.INDEX_MAX
    # m < 2^53 < 2m: the bound Modified Barrett relies on (Section 3.1).
    assert g["modulus"] < g["two53"] < 2 * g["modulus"]
    # The oracle's multiplier is 2^53 (Eq. 3): one step from z = 1.
    assert orc.step(1) == pow(2, g["multiplier_exponent"], M)


def _alpha_floor(nbits):
    """floor(2^nbits * alpha_{2,3}) exactly, from the defining series."""
    s = Fraction(0)
    k = 1
    while 3 ** k <= nbits + 400:
        s += Fraction(1, 3 ** k * 2 ** (3 ** k))
        k += 1
    s += Fraction(1, 3 ** k * 2 ** (3 ** k))  # first omitted term kept too
    return (s.numerator << nbits) // s.denominator


def test_eq1_and_digit_sum_match_alpha_expansion():
    """Eq. 1: x_n = (2^(n-3^e) floor(3^e/2) mod 3^e)/3^e + eps; its top 53 bits
    are alpha's bits n+1..n+53 away from the next power of three."""
    nbits = 3 ** 8 + 200
    a_floor = _alpha_floor(nbits)
    mask = (1 << 53) - 1
    checked = 0
    for e in range(1, 8):
        m = 3 ** e
        for n in range(m, 3 ** (e + 1) - 117):
            bits = (a_floor >> (nbits - n - 53)) & mask
            s = orc.g_index_state(n, e)
            assert (s << 53) // m == bits, (e, n)
            assert (orc.g_digit_sum(n, e) << 53) // m == bits, (e, n)
            checked += 1
    assert checked > 6000


def test_floor_half_identity():
    """sum_{k=1}^{e} 3^(e-k) 2^(3^e-3^k) == floor(3^e/2) (mod 3^e): the constant
    of Eq. 2 is the alpha digit sum at n = 3^e."""
    for e in range(1, 34):
        m = 3 ** e
        acc = sum(3 ** (e - k) * pow(2, 3 ** e - 3 ** k, m) for k in range(1, e + 1)) % m
        assert acc == m // 2
        assert orc.g_index_state(m, e) == m // 2
        if e <= 20:
            assert orc.g_digit_sum(m, e) == m // 2


def test_eq2_equals_digit_sum_full_scale():
    """At modulus 3^33, Eq. 2 at position n equals the truncated alpha sum."""
    rng = random.Random(11)
    seeds = [wl.INDEX_MIN, wl.INDEX_MAX, wl.plain_bulk().index]
    seeds += [rng.randint(wl.INDEX_MIN, wl.INDEX_MAX) for _ in range(20)]
    for a in seeds:
        for k in (0, 1, 2, 3, 1000, 12345):
            n = a + 53 * k
            assert orc.index_state(n) == orc.digit_sum(n)


def test_generated_states_are_alpha_digit_sums():
    """z_k after seed a equals the alpha digit sum at position a + 53k."""
    for a in (wl.INDEX_MIN, wl.plain_bulk().index, 8_000_000_000_000_001):
        z0 = orc.seed(a)
        assert z0 == orc.digit_sum(a)
        zs, zn = orc.gen(z0, 2000, "u64")
        for k in list(range(1, 40)) + [257, 1024, 1999, 2000]:
            assert int(zs[k - 1]) == orc.digit_sum(a + 53 * k), (a, k)
        assert zn == int(zs[-1])


def test_powmod_matches_python_pow():
    rng = random.Random(5)
    for _ in range(2000):
        m = rng.choice([M, 3 ** rng.randint(1, 33), rng.randint(2, 2 ** 63)])
        b = rng.randrange(0, 2 ** 64)
        e = rng.randrange(0, 2 ** 64)
        assert orc.powmod(b, e, m) == pow(b, e, m)
        a2 = rng.randrange(0, m)
        assert orc.mulmod(a2, b % m, m) == a2 * (b % m) % m


def test_period_is_two_times_three_to_32():
    assert orc.powmod(2, P, M) == 1
    assert orc.powmod(2, P // 2, M) != 1
    assert orc.powmod(2, P // 3, M) != 1
    # The multiplier 2^53 has the same order because gcd(53, P) = 1.
    z = orc.seed(wl.INDEX_MIN)
    assert orc.skip(z, P) == z
    assert orc.skip(z, P // 2) != z
    assert orc.skip(z, P // 3) != z


@pytest.mark.parametrize("e", [4, 5, 6, 7, 8, 9])
def test_full_cycle_small_analogue(e):
    """Modulus 3^e, multiplier 2^53 mod 3^e: one cycle through every unit."""
    m = orc.g_modulus(e)
    assert m == 3 ** e
    if e == 5:
        assert pow(2, 53, m) == 41 and orc.g_step(1, e, 53) == 41
    seen = set()
    z = 1
    while True:
        seen.add(z)
        z = orc.g_step(z, e, 53)
        if z == 1:
            break
        assert z not in seen
    units = {u for u in range(1, m) if u % 3}
    assert len(seen) == 2 * 3 ** (e - 1) == len(units)
    assert seen == units


def test_skip_equals_stepping():
    z = orc.seed(wl.plain_bulk().index)
    zs, _ = orc.gen(z, 100_000, "u64")
    for k in [1, 2, 3, 63, 64, 65, 4095, 4096, 65537, 99_999, 100_000]:
        assert orc.skip(z, k) == int(zs[k - 1])
    assert orc.skip(z, 0) == z
    w = z
    for k in range(1, 200):
        w = orc.step(w)
        assert orc.skip(z, k) == w == int(zs[k - 1])


def test_skip_huge_offsets_via_period():
    """skip(seed(a), k) = 2^((a - 3^33 + 53 k) mod P) * floor(3^33/2) mod 3^33."""
    rng = random.Random(7)
    ks = [0, 1, P - 1, P, P + 1, 2 ** 64 - 1, 2 ** 63, 53 * P]
    ks += [rng.randrange(0, 2 ** 64) for _ in range(300)]
    for a in (wl.INDEX_MIN, wl.plain_bulk().index):
        z0 = orc.seed(a)
        for k in ks:
            k = k % 2 ** 64
            want = pow(2, (a - M + 53 * k) % P, M) * H % M
            assert orc.skip(z0, k) == want, (a, k)


def test_chaining_and_zero_count():
    z = orc.seed(wl.INDEX_MIN)
    whole, zw = orc.gen(z, 5000, "f64")
    a, za = orc.gen(z, 1234, "f64")
    b, zb = orc.gen(za, 5000 - 1234, "f64")
    assert np.array_equal(np.concatenate([a, b]).view(np.uint64), whole.view(np.uint64))
    assert zb == zw
    e, ze = orc.gen(z, 0, "u64")
    assert e.size == 0 and ze == z


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_parallel_partition_equals_serial(threads):
    z = orc.seed(wl.plain_bulk().index)
    for kind in ("u64", "f64"):
        s, zs = orc.gen(z, 100_003, kind)
        p, zp = orc.gen(z, 100_003, kind, threads=threads)
        assert np.array_equal(s.view(np.uint64), p.view(np.uint64))
        assert zs == zp


def test_f64_is_rounded_product_with_rounded_reciprocal():
    """Reading of Algorithm BB step 3 / the listings: RN(z * RN(1/3^33))."""
    r = Fraction(float(Fraction(1, M)))  # RN(1/m) by exact rational rounding
    assert float(r) == 1.0 / 5559060566555523.0
    rng = random.Random(3)
    zs = [1, 2, 4, M - 1, M - 2, H, H + 1] + [rng.randrange(1, M) for _ in range(20000)]
    zs = [z for z in zs if z % 3]
    differs = 0
    for z in zs:
        got = orc.to_f64(z)
        want = float(Fraction(z) * r)
        assert got == want, z
        assert 0.0 < got < 1.0
        exact = Fraction(z, M)
        assert abs(Fraction(got) - exact) <= exact * Fraction(1, 2 ** 52)
        differs += got != float(exact)
    # A measurable share of states is not the correctly rounded quotient.
    assert 0.01 < differs / len(zs) < 0.05


def test_f64_stream_matches_u64_stream():
    z = orc.seed(wl.INDEX_MIN)
    u, zu = orc.gen(z, 4096, "u64")
    f, zf = orc.gen(z, 4096, "f64")
    assert zu == zf
    assert all(orc.to_f64(int(x)) == y for x, y in zip(u[:512], f[:512]))


def test_seed_range_and_distinct_states():
    assert orc.seed(wl.INDEX_MIN) == orc.digit_sum(wl.INDEX_MIN)
    assert orc.seed(wl.INDEX_MAX) == orc.index_state(wl.INDEX_MAX)
    for bad in (0, 3 ** 33, wl.INDEX_MIN - 1, wl.INDEX_MAX + 1, 2 ** 64 - 1):
        with pytest.raises(ValueError):
            orc.seed(bad)
    rng = random.Random(9)
    idx = {rng.randint(wl.INDEX_MIN, wl.INDEX_MAX) for _ in range(3000)}
    states = {orc.seed(a) for a in idx}
    assert len(states) == len(idx)
    assert all(s % 3 and 0 < s < M for s in states)


def test_modified_barrett_comparator():
    """Section 3.1's Modified Barrett step equals Eq. 3 for every unit state."""
    g = _golden()
    assert g["mu"] == 2 ** 106 // M
    rng = random.Random(13)
    zs = [1, 2, 4, 5, M - 1, M - 2, M - 4, H, H + 1, 2 ** 52, 2 ** 52 + 1]
    zs += [rng.randrange(1, M) for _ in range(100_000)]
    # states whose 2^53 z is just above / below a multiple of m
    inv = pow(2 ** 53, -1, M)
    zs += [(r * inv) % M for r in (1, 2, 4, M - 1, M - 2, M - 4, H, H + 2)]
    for z in zs:
        if z % 3 == 0:
            continue
        assert orc.modbarrett_step(z) == pow(2, 53, M) * z % M, z
    z = orc.seed(wl.INDEX_MIN)
    mb, zmb = orc.gen_f64_modbarrett(z, 10_000)
    ref, zr = orc.gen(z, 10_000, "f64")
    assert np.array_equal(mb.view(np.uint64), ref.view(np.uint64)) and zmb == zr


def test_workload_recipes():
    pb = wl.plain_bulk()
    assert wl.INDEX_MIN <= pb.index <= wl.INDEX_MAX
    assert (pb.count_f64, pb.count_u64) == (1 << 30, 1 << 28)
    off = wl.skip_offsets()
    assert off.size == 65536 and int(off.max()) == P - 1 and int(off.min()) == 0
    assert int((off >= P - 4096).sum()) >= 64
    b = wl.batched()
    assert b.lengths.size == 10000 and int(b.lengths.min()) >= 1
    assert int(b.lengths.max()) <= 2 ** 22
    assert int(b.indices.min()) >= wl.INDEX_MIN and int(b.indices.max()) <= wl.INDEX_MAX
