"""CPU oracle for the alpha_{2,3} normal-number LCG (Beliakov et al., Section 2).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its binding) never imports this package, and this package never imports the
product path.

This module is argument marshalling over ``liborc.so`` (plain C with 128-bit
integer products, ``nn_oracle.c``); numpy arrays carry the outputs.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

#: 3^33, the modulus of Eqs. 2-3.
MOD = 5559060566555523
#: Seed range of Algorithm BB step 1 (inclusive).
INDEX_MIN = MOD + 100
INDEX_MAX = 2 ** 53

_u64 = ctypes.c_uint64
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build  # the oracle library is built on demand
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "orc_mulmod": (_u64, [_u64, _u64, _u64]),
        "orc_powmod": (_u64, [_u64, _u64, _u64]),
        "orc_seed": (ctypes.c_int, [_u64, ctypes.POINTER(_u64)]),
        "orc_step": (_u64, [_u64]),
        "orc_skip": (_u64, [_u64, _u64]),
        "orc_index_state": (_u64, [_u64]),
        "orc_digit_sum": (_u64, [_u64]),
        "orc_to_f64": (ctypes.c_double, [_u64]),
        "orc_gen_u64": (_u64, [_u64, _u64, ctypes.c_void_p]),
        "orc_gen_f64": (_u64, [_u64, _u64, ctypes.c_void_p]),
        "orc_gen_par": (_u64, [_u64, _u64, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
        "orc_max_threads": (ctypes.c_int, []),
        "orc_g_modulus": (_u64, [ctypes.c_int]),
        "orc_g_step": (_u64, [_u64, ctypes.c_int, ctypes.c_int]),
        "orc_g_index_state": (_u64, [_u64, ctypes.c_int]),
        "orc_g_digit_sum": (_u64, [_u64, ctypes.c_int]),
        "orc_e40_seed": (ctypes.c_int, [_u64, ctypes.POINTER(_u64)]),
        "orc_e40_step": (_u64, [_u64]),
        "orc_e40_skip": (_u64, [_u64, _u64]),
        "orc_e40_to_f64": (ctypes.c_double, [_u64]),
        "orc_e40_gen_u64": (_u64, [_u64, _u64, ctypes.c_void_p]),
        "orc_e40_gen_f64": (_u64, [_u64, _u64, ctypes.c_void_p]),
        "orc_modbarrett_step": (_u64, [_u64]),
        "orc_gen_f64_modbarrett": (_u64, [_u64, _u64, ctypes.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def mulmod(a, b, m):
    return int(_load().orc_mulmod(a, b, m))


def powmod(b, e, m):
    return int(_load().orc_powmod(b, e, m))


def seed(index):
    """Eq. 2 state for a starting index; raises ValueError outside [3^33+100, 2^53]."""
    z = _u64(0)
    if index < 0 or index >= 2 ** 64 or _load().orc_seed(index, ctypes.byref(z)) != 0:
        raise ValueError("seed index %r outside [3^33+100, 2^53]" % (index,))
    return int(z.value)


def step(z):
    """Eq. 3: 2^53 z mod 3^33."""
    return int(_load().orc_step(z))


def skip(z, k):
    """State k steps after z (k any 64-bit count)."""
    return int(_load().orc_skip(z, k))


def index_state(n):
    return int(_load().orc_index_state(n))


def digit_sum(n):
    return int(_load().orc_digit_sum(n))


def to_f64(z):
    return float(_load().orc_to_f64(z))


def gen(z, n, kind="f64", threads=1):
    """Emit z_1..z_n after state z; returns (array, z_n).

    ``kind`` is "u64" (raw states) or "f64" (variates).  ``threads`` > 1 (or
    0 for all) uses the OpenMP skip-ahead partition instead of one chain.
    """
    dtype = np.uint64 if kind == "u64" else np.float64
    out = np.empty(int(n), dtype=dtype)
    ptr = out.ctypes.data_as(ctypes.c_void_p)
    lib = _load()
    if threads == 1:
        fn = lib.orc_gen_u64 if kind == "u64" else lib.orc_gen_f64
        zn = fn(z, n, ptr)
    else:
        zn = lib.orc_gen_par(z, n, ptr, 0 if kind == "u64" else 1, int(threads))
    return out, int(zn)


def gen_into(z, out, threads=0):
    """Fill a preallocated uint64/float64 numpy array; returns z_n."""
    kind = 0 if out.dtype == np.uint64 else 1
    assert out.dtype in (np.uint64, np.float64) and out.flags.c_contiguous
    return int(_load().orc_gen_par(z, out.size, out.ctypes.data_as(ctypes.c_void_p),
                                   kind, int(threads)))


def max_threads():
    return int(_load().orc_max_threads())


def g_modulus(e):
    return int(_load().orc_g_modulus(e))


def g_step(z, e, b):
    return int(_load().orc_g_step(z, e, b))


def g_index_state(n, e):
    return int(_load().orc_g_index_state(n, e))


def g_digit_sum(n, e):
    return int(_load().orc_g_digit_sum(n, e))


def modbarrett_step(z):
    return int(_load().orc_modbarrett_step(z))


def gen_f64_modbarrett(z, n):
    out = np.empty(int(n), dtype=np.float64)
    zn = _load().orc_gen_f64_modbarrett(z, n, out.ctypes.data_as(ctypes.c_void_p))
    return out, int(zn)


# ------------------------------------------------------------ modulus 3^40 --
#: 3^40, the larger modulus Section 2 names for a longer period.
E40_MOD = 3 ** 40
E40_INDEX_MIN = E40_MOD + 100
E40_INDEX_MAX = 2 ** 64 - 1


def e40_seed(index):
    """Eq. 2 at modulus 3^40; ValueError outside [3^40+100, 2^64-1]."""
    z = _u64(0)
    if index < 0 or index >= 2 ** 64 or _load().orc_e40_seed(index, ctypes.byref(z)) != 0:
        raise ValueError("seed index %r outside [3^40+100, 2^64-1]" % (index,))
    return int(z.value)


def e40_step(z):
    return int(_load().orc_e40_step(z))


def e40_skip(z, k):
    return int(_load().orc_e40_skip(z, k))


def e40_to_f64(z):
    return float(_load().orc_e40_to_f64(z))


def e40_gen(z, n, kind="u64"):
    """Serial outputs z_1..z_n after z at modulus 3^40 (numpy) and z_n."""
    if kind == "u64":
        out = np.empty(n, dtype=np.uint64)
        zn = _load().orc_e40_gen_u64(z, n, out.ctypes.data_as(ctypes.c_void_p))
    else:
        out = np.empty(n, dtype=np.float64)
        zn = _load().orc_e40_gen_f64(z, n, out.ctypes.data_as(ctypes.c_void_p))
    return out, int(zn)
