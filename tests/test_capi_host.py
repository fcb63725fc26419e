"""CPU tests of the C ABI (include/nn.h): exports, host-side arithmetic,
argument validation that happens before any device call, and the host build
of every step-loop reduction.  Expected values come from the oracle or from
Python's own integers, never from the library."""
import ctypes
import os
import random
import re

import numpy as np
import pytest

import oracle as orc
import paper_1206_1187_amd as nn
from paper_1206_1187_amd import _native
from paper_1206_1187_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M = 3 ** 33
P = 2 * 3 ** 32


def _declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:int|const\s+char\s*\*)\s*(nn_\w+)\s*\(", text, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 10 and "nn_generate" in names and "nn_seed" in names
    lib = _native.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows the signature of each declared entry point
    assert set(names) <= set(_native.SIGNATURES), set(names) - set(_native.SIGNATURES)


def test_header_constants_match_paper():
    text = open(os.path.join(ROOT, "include", "nn.h")).read()
    consts = dict(re.findall(r"#define\s+(NN_\w+)\s+(\d+)ULL", text))
    assert int(consts["NN_MODULUS"]) == 3 ** 33
    assert int(consts["NN_PERIOD"]) == 2 * 3 ** 32
    assert int(consts["NN_INDEX_MIN"]) == 3 ** 33 + 100
    assert int(consts["NN_INDEX_MAX"]) == 2 ** 53


def test_header_flags_match_binding():
    """Every NN_CFG_* / NN_BATCH_* / NN_SERVER_* flag and the debug selector
    the binding uses has the value include/nn.h gives it."""
    text = open(os.path.join(ROOT, "include", "nn.h")).read()
    flags = {k: int(v) for k, v in re.findall(r"#define\s+(NN_\w+)\s+(\d+)u?\b", text)}
    names = [n for n in dir(_native) if n.startswith(("NN_CFG_", "NN_BATCH_", "NN_SERVER_",
                                                       "NN_DEBUG_"))]
    assert "NN_CFG_NONTEMPORAL_STORES" in names
    for n in names:
        assert n in flags and flags[n] == getattr(_native, n), n


def test_make_cfg_store_policy_and_layout_flags():
    """make_cfg's temporal argument: None keeps the layout default (no flag),
    True and False set the explicit flags; the layout names set theirs."""
    assert nn.make_cfg().flags == 0
    assert nn.make_cfg(temporal=True).flags == _native.NN_CFG_TEMPORAL_STORES
    assert nn.make_cfg(temporal=False).flags == _native.NN_CFG_NONTEMPORAL_STORES
    c = nn.make_cfg(layout="flat", unroll=4, occupancy=4)
    assert c.flags == _native.NN_CFG_FLAT and c.unroll == 4 and c.occupancy == 4
    assert nn.make_cfg(layout="rows", temporal=False).flags == (
        _native.NN_CFG_ROWS | _native.NN_CFG_NONTEMPORAL_STORES)
    with pytest.raises(nn.NNError):
        nn.make_cfg(layout="diagonal")


def test_version_and_strerror():
    assert "gfx950" in nn.version()
    lib = _native.lib()
    for st in range(6):
        assert lib.nn_strerror(st)
    assert lib.nn_strerror(99) == b"unknown status"


def test_seed_matches_oracle():
    rng = random.Random(1)
    idx = [wl.INDEX_MIN, wl.INDEX_MIN + 1, wl.INDEX_MAX, wl.INDEX_MAX - 1, wl.plain_bulk().index]
    idx += [rng.randint(wl.INDEX_MIN, wl.INDEX_MAX) for _ in range(3000)]
    for a in idx:
        assert nn.seed(a) == orc.seed(a), a


@pytest.mark.parametrize("bad", [0, 1, 3 ** 33, wl.INDEX_MIN - 1, wl.INDEX_MAX + 1, 2 ** 64 - 1])
def test_seed_rejects_out_of_range(bad):
    with pytest.raises(nn.NNError) as ei:
        nn.seed(bad)
    assert ei.value.status == _native.NN_EINVAL


def test_seed_null_pointer():
    assert _native.lib().nn_seed(wl.INDEX_MIN, None) == _native.NN_EINVAL


def test_skip_matches_oracle():
    rng = random.Random(2)
    z = orc.seed(wl.plain_bulk().index)
    ks = [0, 1, 2, 255, 256, 257, 65535, 65536, 2 ** 24, P - 1, P, P + 1, 2 ** 56, 2 ** 63,
          2 ** 64 - 1]
    ks += [rng.randrange(0, 2 ** 64) for _ in range(3000)]
    for k in ks:
        assert nn.skip(z, k) == orc.skip(z, k), k
    states = [1, 2, M - 1, M - 2] + [orc.seed(rng.randint(wl.INDEX_MIN, wl.INDEX_MAX))
                                     for _ in range(200)]
    for s in states:
        k = rng.randrange(0, 2 ** 64)
        assert nn.skip(s, k) == orc.skip(s, k)


@pytest.mark.parametrize("bad", [0, 3, 6, M, M + 1, 2 ** 53, 2 ** 64 - 1, 3 * 12345])
def test_skip_rejects_non_units(bad):
    with pytest.raises(nn.NNError) as ei:
        nn.skip(bad, 5)
    assert ei.value.status == _native.NN_EINVAL


def _adversarial_pairs(rng, n):
    """Pairs (z, v) whose product residue is at the edges of every reduction:
    residues 1, 2, m-1, m-2 and around m/2 (ties of the quotient rounding)."""
    a, b = [], []
    targets = [1, 2, 4, M - 1, M - 2, M - 4, M // 2, M // 2 + 1, M // 2 - 1, M // 2 + 2,
               M // 2 + 3, M // 2 - 2]
    targets = [t for t in targets if t % 3]
    for _ in range(n):
        z = rng.randrange(1, M)
        while z % 3 == 0:
            z = rng.randrange(1, M)
        r = rng.choice(targets)
        v = r * pow(z, -1, M) % M
        a.append(z)
        b.append(v)
    fixed = [1, 2, 4, M - 1, M - 2, M - 4, M // 2, M // 2 + 1, 2 ** 52 + 1, 2 ** 52 - 1]
    fixed = [x for x in fixed if x % 3]
    for x in fixed:
        for y in fixed:
            a.append(x)
            b.append(y)
    return a, b


@pytest.mark.parametrize("variant", ["fp64", "barrett", "shoup", "montgomery", "device"])
def test_host_build_of_reductions_is_exact(variant):
    """Every reduction, and the public device header's nn_dev_mulmod
    ("device"), on random and adversarial pairs against Python integers."""
    rng = random.Random(hash(variant) & 0xffff)
    a, b = _adversarial_pairs(rng, 20000)
    r = np.random.default_rng(7)
    za = r.integers(1, M, 200000, dtype=np.int64)
    zb = r.integers(1, M, 200000, dtype=np.int64)
    keep = (za % 3 != 0) & (zb % 3 != 0)
    a = np.concatenate([np.array(a, dtype=np.uint64), za[keep].astype(np.uint64)])
    b = np.concatenate([np.array(b, dtype=np.uint64), zb[keep].astype(np.uint64)])
    got = nn.debug_mulmod(variant, a, b)
    # Expected: the oracle's 128-bit product modulo m on a sample, Python's
    # integers on the rest.
    for i in range(0, a.size, 97):
        assert int(got[i]) == orc.mulmod(int(a[i]), int(b[i]), M)
    want = np.array([int(x) * int(y) % M for x, y in zip(a.tolist(), b.tolist())],
                    dtype=np.uint64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(a[i]), int(b[i]), int(got[i]), int(want[i])) for i in bad[:5]]


def test_host_build_of_modified_barrett_step_is_exact():
    """Section 3.1's Modified Barrett step (2^53 z mod 3^33) on states whose
    residue sits at the edges: 1, 2, m-1, m-2, and on both sides of the
    boundary where the quotient estimate falls one short (residues near
    (2^53 - m) = 0.62 m), plus random states; expected from Python's
    integers, a sample also from the oracle's own comparator."""
    M53 = pow(2, 53, M)
    inv = pow(M53, -1, M)
    rng = random.Random(53)
    edge = [1, 2, 4, M - 1, M - 2, M - 4, 2 ** 53 - M, 2 ** 53 - M - 1, 2 ** 53 - M + 1]
    edge += [int(M * f) + d for f in (0.6172, 0.6203, 0.5, 0.25) for d in range(-40, 41)]
    zs = [r * inv % M for r in edge if r % 3]
    zs += [rng.randrange(1, M) for _ in range(100000)]
    zs = np.array([z for z in zs if z % 3], dtype=np.uint64)
    got = nn.debug_mulmod("modbarrett", zs, np.full(zs.size, M53, dtype=np.uint64))
    want = np.array([(int(z) << 53) % M for z in zs.tolist()], dtype=np.uint64)
    assert np.array_equal(got, want)
    for i in range(0, zs.size, 101):
        assert int(got[i]) == orc.modbarrett_step(int(zs[i]))
    with pytest.raises(nn.NNError):  # only the multiplier 2^53
        nn.debug_mulmod("modbarrett", [5], [7])


def test_debug_mulmod_rejects_non_units():
    with pytest.raises(nn.NNError):
        nn.debug_mulmod("fp64", [3], [5])
    with pytest.raises(nn.NNError):
        nn.debug_mulmod(9, [1], [1])


def test_generate_validation_before_device():
    """Errors that must be reported before any HIP call is made."""
    lib = _native.lib()
    st = ctypes.c_uint64(orc.seed(wl.INDEX_MIN))
    buf = ctypes.create_string_buffer(64)
    aligned = ctypes.addressof(buf) + (-ctypes.addressof(buf)) % 8
    # NULL state pointer
    assert lib.nn_generate(None, 8, ctypes.c_void_p(aligned), 0, None) == _native.NN_EINVAL
    # bad kind
    assert lib.nn_generate(ctypes.byref(st), 8, ctypes.c_void_p(aligned), 7, None) == _native.NN_EINVAL
    # invalid states
    for bad in (0, 3, M, 2 ** 64 - 1):
        s2 = ctypes.c_uint64(bad)
        assert lib.nn_generate(ctypes.byref(s2), 8, ctypes.c_void_p(aligned), 1, None) == _native.NN_EINVAL
        assert s2.value == bad
    # count 0 is a no-op even with a NULL output
    s3 = ctypes.c_uint64(st.value)
    assert lib.nn_generate(ctypes.byref(s3), 0, None, 1, None) == _native.NN_OK
    assert s3.value == st.value
    # NULL and misaligned outputs, count overflow
    assert lib.nn_generate(ctypes.byref(st), 8, None, 1, None) == _native.NN_EINVAL
    assert lib.nn_generate(ctypes.byref(st), 8, ctypes.c_void_p(aligned + 4), 1, None) == _native.NN_EINVAL
    assert lib.nn_generate(ctypes.byref(st), 2 ** 61, ctypes.c_void_p(aligned), 1, None) == _native.NN_ERANGE
    assert st.value == orc.seed(wl.INDEX_MIN)
    lib.nn_generate(ctypes.byref(st), 8, ctypes.c_void_p(aligned + 4), 1, None)
    assert b"aligned" in lib.nn_last_error()
    # fill: same pointer rules
    assert lib.nn_fill(0, None, 0, None, None) == _native.NN_OK
    assert lib.nn_fill(8, ctypes.c_void_p(aligned + 4), 0, None, None) == _native.NN_EINVAL


def test_batch_plan_validation_before_device():
    """Batch-plan configurations that are refused before any HIP call: the
    residency cap belongs to the chunked kernel and lies in [2, 16]."""
    lib = _native.lib()
    h = ctypes.c_void_p()
    for flags, occ in [(0, 4), (_native.NN_BATCH_INTERLEAVED, 4),
                       (_native.NN_BATCH_CHUNKS, 1), (_native.NN_BATCH_CHUNKS, 17)]:
        cfg = _native.BatchCfg(0, 0, 0, 0, flags, occ)
        assert lib.nn_batch_plan_create(1, 8, 1 << 20, ctypes.byref(cfg),
                                        ctypes.byref(h)) == _native.NN_EINVAL
        assert b"occupancy" in lib.nn_last_error()
        assert not h.value


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(_native, "LIB_PATH", "/nonexistent/libnn.so")
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(_native.NativeLibraryMissing):
        nn.seed(wl.INDEX_MIN)


def test_dev_mult_pow_is_the_power_and_its_quotient():
    """nn_dev_mult_pow(k): v = (2^53)^(k mod P) mod 3^33 (Python integers)
    and qh + ql = v / 3^33 to double-double accuracy (exact rationals), far
    inside what nn_dev_mulmod needs: its remainder stays in (-3^33, 3^33)
    while |q - v z / 3^33| < 1, i.e. while z times this error stays below a
    quarter (z < 2^53)."""
    from fractions import Fraction
    mult = pow(2, 53, M)
    ks = [0, 1, 2, 53, 1023, 1 << 20, P - 1, P, P + 1, 2 ** 63, 2 ** 64 - 1]
    rng = random.Random(5)
    ks += [rng.getrandbits(64) for _ in range(20)]
    for k in ks:
        v, qh, ql = nn.dev_mult_pow(k)
        want = pow(mult, k % P, M)
        assert v == float(want) and int(v) == want, k
        err = abs(Fraction(qh) + Fraction(ql) - Fraction(want, M))
        # 106 bits of floor(v 2^128 / 3^33) 2^-128: relative 2^-105 or absolute 2^-128
        assert err <= Fraction(want, M) / 2 ** 105 + Fraction(1, 2 ** 128), k
        assert abs(ql) <= abs(qh) * 2.0 ** -52, k
    with pytest.raises(nn.NNError):
        _native.check(_native.lib().nn_dev_mult_pow(1, None))
