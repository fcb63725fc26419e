"""CPU tests of the modulus-3^40 C ABI (nn_e40_*): seeding, skip-ahead, the
host build of the Montgomery step and the argument checks made before any
device call.  Expected values from the oracle or Python's integers."""
import ctypes
import random

import numpy as np
import pytest

import oracle as orc
import paper_1206_1187_amd as nn
from paper_1206_1187_amd import _native

M = 3 ** 40
P = 2 * 3 ** 39


def test_e40_seed_matches_oracle():
    rng = random.Random(1)
    idx = [nn.E40_INDEX_MIN, nn.E40_INDEX_MAX, nn.E40_INDEX_MIN + 1]
    idx += [rng.randint(nn.E40_INDEX_MIN, nn.E40_INDEX_MAX) for _ in range(200)]
    for a in idx:
        assert nn.e40_seed(a) == orc.e40_seed(a)
    for bad in (0, M, nn.E40_INDEX_MIN - 1):
        with pytest.raises(nn.NNError):
            nn.e40_seed(bad)


def test_e40_skip_matches_pow():
    rng = random.Random(2)
    z = orc.e40_seed(nn.E40_INDEX_MIN)
    for k in [0, 1, 2, 53, P - 1, P, P + 5, 2 ** 64 - 1] + [rng.getrandbits(64) for _ in range(100)]:
        assert nn.e40_skip(z, k) == z * pow(2 ** 53, k, M) % M
    for bad in (0, 3, M, M + 1, 2 ** 64 - 1):
        with pytest.raises(nn.NNError):
            nn.e40_skip(bad, 1)


def test_e40_host_build_of_montgomery_step_is_exact():
    """Random pairs, and pairs whose product residue is at the edges (1, 2,
    m-1, m-2, m/2), where the 129-bit intermediate sum and the final
    correction are exercised."""
    rng = random.Random(3)
    a, b = [], []
    for _ in range(20000):
        x = rng.randrange(1, M)
        while x % 3 == 0:
            x = rng.randrange(1, M)
        r = rng.choice([1, 2, 4, M - 1, M - 2, M - 4, M // 2, M // 2 + 1, 2 ** 64 - M])
        if r % 3 == 0:
            r += 1
        a.append(x)
        b.append(r * pow(x, -1, M) % M)
    for _ in range(100000):
        x, y = rng.randrange(1, M), rng.randrange(1, M)
        if x % 3 and y % 3:
            a.append(x)
            b.append(y)
    fixed = [1, 2, M - 1, M - 2, 2 ** 63 + 1, 2 ** 64 - M + 1, M // 2]
    fixed = [v for v in fixed if v % 3]
    for x in fixed:
        for y in fixed:
            a.append(x)
            b.append(y)
    want = np.array([x * y % M for x, y in zip(a, b)], dtype=np.uint64)
    for mulmod in ("montgomery", "fp64"):
        got = nn.e40_debug_mulmod(a, b, mulmod)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, [(mulmod, a[i], b[i], int(got[i])) for i in bad[:5]]
        with pytest.raises(nn.NNError):
            nn.e40_debug_mulmod([3], [5], mulmod)
    with pytest.raises(nn.NNError):
        nn.e40_debug_mulmod([1], [1], "barrett")


def test_e40_host_build_of_limb_step_at_limb_edges():
    """The FP64 step splits operands into base-3^20 limbs: operands whose
    limbs sit at 0, 1, B/2 and B - 1 (carries into and out of the high
    limb), and multipliers of the generator itself (2^53 and its powers)."""
    B = 3 ** 20
    rng = random.Random(5)
    limbs = [0, 1, 2, B // 2, B // 2 + 1, B - 2, B - 1]
    vals = sorted({hi * B + lo for hi in limbs for lo in limbs if 0 < hi * B + lo < M})
    vals = [v for v in vals if v % 3]
    mults = vals + [pow(2 ** 53, k, M) for k in (1, 2, 3, 1024, 2 ** 25, rng.randrange(M))]
    a = [x for x in vals for _ in mults]
    b = [y for _ in vals for y in mults]
    want = np.array([x * y % M for x, y in zip(a, b)], dtype=np.uint64)
    assert np.array_equal(nn.e40_debug_mulmod(a, b, "fp64"), want)


def test_e40_generate_validation_before_device():
    lib = _native.lib()
    buf = (ctypes.c_uint64 * 64)()
    aligned = (ctypes.addressof(buf) + 15) // 16 * 16
    st = ctypes.c_uint64(orc.e40_seed(nn.E40_INDEX_MIN))
    assert lib.nn_e40_generate(None, 8, ctypes.c_void_p(aligned), 0, None) == _native.NN_EINVAL
    assert lib.nn_e40_generate(ctypes.byref(st), 8, ctypes.c_void_p(aligned), 5, None) == _native.NN_EINVAL
    for badstate in (0, 3, M, 2 ** 64 - 1):
        s2 = ctypes.c_uint64(badstate)
        assert lib.nn_e40_generate(ctypes.byref(s2), 8, ctypes.c_void_p(aligned), 1, None) == _native.NN_EINVAL
        assert s2.value == badstate
    s3 = ctypes.c_uint64(st.value)
    assert lib.nn_e40_generate(ctypes.byref(s3), 0, None, 1, None) == _native.NN_OK
    assert s3.value == st.value
    assert lib.nn_e40_generate(ctypes.byref(st), 8, None, 1, None) == _native.NN_EINVAL
    assert lib.nn_e40_generate(ctypes.byref(st), 8, ctypes.c_void_p(aligned + 4), 1, None) == _native.NN_EINVAL
    assert lib.nn_e40_generate(ctypes.byref(st), 2 ** 61, ctypes.c_void_p(aligned), 1, None) == _native.NN_ERANGE
    assert st.value == orc.e40_seed(nn.E40_INDEX_MIN)
