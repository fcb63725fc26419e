"""The public device header (include/nn_device.h) used from a consumer
kernel of its own (tests/devapi/example.hip), as a simulation would use it:
two access patterns against the oracle, bit for bit."""
import ctypes
import os

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402
from paper_1206_1187_amd import _native  # noqa: E402

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "devapi", "libdevapi_example.so")


@pytest.fixture(scope="module")
def example():
    assert torch.cuda.is_available()
    nn.init(0)
    assert os.path.exists(LIB), "build the example first (tests/devapi/build.py, run by build())"
    lib = ctypes.CDLL(LIB)
    lib.example_generate.restype = ctypes.c_int
    lib.example_generate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_void_p, _native.DevMult, ctypes.c_void_p,
                                     ctypes.c_void_p]
    return lib


def _mult(k):
    return _native.DevMult(*nn.dev_mult_pow(k))


@pytest.mark.parametrize("mode,param", [(0, 1), (0, 1000), (0, 65536), (1, 1), (1, 7), (1, 4096)])
def test_consumer_kernel_with_public_header(example, mode, param):
    z0 = orc.seed(wl.INDEX_MIN + 777)
    count = 300_001
    ref, _ = orc.gen(z0, count, "f64", threads=0)
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    table = nn.dev_skip_table()
    mult = _mult(param) if mode == 0 else _mult(1)
    rc = example.example_generate(mode, z0, count, param, table, mult, out.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    got = out.view(torch.int64).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref.view(np.uint64))
