"""MI355X-native alpha_{2,3} normal-number uniform generator.

Python binding over ``libnn.so`` (include/nn.h): argument marshalling only.
Every output value is computed by the HIP kernels; torch supplies device
memory and the current stream.  The generator is Algorithm BB of Beliakov
et al. (Section 2): seed z_0 by Eq. 2 from a starting index, step
z -> 2^53 z mod 3^33 (Eq. 3), variates z * 3^-33.

    import paper_1206_1187_amd as nn
    s = nn.seed(3**33 + 100)
    u, s = nn.generate(s, 1 << 20)          # float64 tensor on cuda, new state
"""
import ctypes

from . import _native
from ._native import (NN_OUT_F64, NN_OUT_U64, LaunchCfg, NativeLibraryMissing, NNError,
                      MULMOD_NAMES)

MODULUS = 5559060566555523
PERIOD = 2 * 3 ** 32
INDEX_MIN = MODULUS + 100
INDEX_MAX = 2 ** 53

__all__ = [
    "seed", "skip", "generate", "generate_into", "fill", "default_cfg", "make_cfg", "BatchPlan",
    "init", "version", "NNError", "NativeLibraryMissing", "MODULUS", "PERIOD",
    "INDEX_MIN", "INDEX_MAX",
]


def version():
    return _native.lib().nn_version().decode()


def seed(index):
    """Eq. 2: state of starting index ``index`` in [3^33+100, 2^53]."""
    out = ctypes.c_uint64(0)
    if not 0 <= int(index) < 2 ** 64:
        raise NNError(_native.NN_EINVAL, "index out of the 64-bit range")
    _native.check(_native.lib().nn_seed(int(index), ctypes.byref(out)))
    return int(out.value)


def skip(state, k):
    """State ``k`` steps after ``state`` (k reduced modulo the period)."""
    out = ctypes.c_uint64(0)
    _native.check(_native.lib().nn_skip(int(state), int(k) % 2 ** 64, ctypes.byref(out)))
    return int(out.value)


def init(device=0):
    _native.check(_native.lib().nn_init(int(device)))


def make_cfg(block=0, grid=0, mulmod=0, unroll=0, temporal=None, width=0, layout=None,
             occupancy=0, ilp=0, address_order=False):
    """Launch configuration (include/nn.h, nn_launch_cfg); ``layout`` is
    None (library default), "flat", "rows", "consecutive" or "paper_strided"
    (the paper's transposed order: out[t + i*T] = element t*E + i).
    ``temporal``: None keeps the layout's default store policy, True asks for
    temporal stores, False for non-temporal ones.  ``address_order``: the
    flat layout's chunks in address order instead of XCD runs
    (NN_CFG_ADDRESS_ORDER)."""
    if isinstance(mulmod, str):
        mulmod = MULMOD_NAMES[mulmod]
    flags = {None: 0, True: _native.NN_CFG_TEMPORAL_STORES,
             False: _native.NN_CFG_NONTEMPORAL_STORES}[temporal]
    if layout == "flat":
        flags |= _native.NN_CFG_FLAT
    elif layout == "rows":
        flags |= _native.NN_CFG_ROWS
    elif layout == "consecutive":
        flags |= _native.NN_CFG_CONSECUTIVE
    elif layout == "paper_strided":
        flags |= _native.NN_CFG_PAPER_STRIDED
    elif layout is not None:
        raise NNError(_native.NN_EINVAL, "layout must be None, 'flat', 'rows', 'consecutive' "
                      "or 'paper_strided'")
    if address_order:
        flags |= _native.NN_CFG_ADDRESS_ORDER
    return LaunchCfg(int(block), int(grid), int(mulmod), int(unroll), flags, int(width),
                     int(occupancy), int(ilp))


def default_cfg(kind, count):
    cfg = LaunchCfg()
    _native.check(_native.lib().nn_default_cfg(_kind(kind), int(count), ctypes.byref(cfg)))
    return cfg


def _kind(kind):
    if kind in (NN_OUT_U64, "u64", "uint64"):
        return NN_OUT_U64
    if kind in (NN_OUT_F64, "f64", "float64"):
        return NN_OUT_F64
    import torch
    if kind == torch.uint64:
        return NN_OUT_U64
    if kind == torch.float64:
        return NN_OUT_F64
    raise NNError(_native.NN_EINVAL, "unknown output kind %r" % (kind,))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def generate_into(state, out, stream=None, cfg=None):
    """Fill the contiguous cuda tensor ``out`` (uint64 or float64) with the
    next ``out.numel()`` outputs after ``state``; returns the new state.
    Asynchronous on ``stream`` (default: torch's current stream)."""
    import torch
    if not out.is_cuda or not out.is_contiguous():
        raise NNError(_native.NN_EINVAL, "out must be a contiguous cuda tensor")
    kind = _kind(out.dtype)
    st = ctypes.c_uint64(int(state))
    with torch.cuda.device(out.device):
        rc = _native.lib().nn_generate_ex(
            ctypes.byref(st), out.numel(), ctypes.c_void_p(out.data_ptr()), kind,
            _stream_handle(stream), ctypes.byref(cfg) if cfg is not None else None)
    _native.check(rc)
    return int(st.value)


def generate(state, count, dtype="f64", device="cuda", stream=None, cfg=None):
    """Allocate and fill ``count`` outputs; returns (tensor, new_state)."""
    import torch
    tdtype = torch.uint64 if _kind(dtype) == NN_OUT_U64 else torch.float64
    out = torch.empty(int(count), dtype=tdtype, device=device)
    return out, generate_into(state, out, stream=stream, cfg=cfg)


def fill(out, value, stream=None, cfg=None, with_start=False):
    """The paper's "Constant" kernel: write ``value`` (a 64-bit pattern) with
    the generator's store pattern; ``with_start`` (flat layout) also makes
    the generator's start-up table loads (NN_FILL_WITH_START)."""
    import torch
    if not out.is_cuda or not out.is_contiguous() or out.element_size() != 8:
        raise NNError(_native.NN_EINVAL, "out must be a contiguous 8-byte cuda tensor")
    if with_start:
        c = _native.LaunchCfg()
        if cfg is not None:
            ctypes.pointer(c)[0] = cfg
        c.flags |= _native.NN_FILL_WITH_START
        cfg = c
    with torch.cuda.device(out.device):
        rc = _native.lib().nn_fill(out.numel(), ctypes.c_void_p(out.data_ptr()),
                                   int(value) % 2 ** 64, _stream_handle(stream),
                                   ctypes.byref(cfg) if cfg is not None else None)
    _native.check(rc)


def consume(state, count, kind="u64", result=None, stream=None, cfg=None):
    """The fused consumer: add the sum of the next ``count`` outputs (raw
    states modulo 2^64 for "u64", variates for "f64") to the one-element
    cuda tensor ``result`` (allocated and zeroed when None).  Returns
    (result, new_state)."""
    import torch
    k = _kind(kind)
    if result is None:
        result = torch.zeros(1, dtype=torch.int64 if k == NN_OUT_U64 else torch.float64,
                             device="cuda")
    st = ctypes.c_uint64(int(state))
    with torch.cuda.device(result.device):
        rc = _native.lib().nn_consume(ctypes.byref(st), int(count), k,
                                      ctypes.c_void_p(result.data_ptr()), _stream_handle(stream),
                                      ctypes.byref(cfg) if cfg is not None else None)
    _native.check(rc)
    return result, int(st.value)


E40_MODULUS = 3 ** 40
E40_INDEX_MIN = E40_MODULUS + 100
E40_INDEX_MAX = 2 ** 64 - 1


def e40_seed(index):
    """Eq. 2 at modulus 3^40 (include/nn.h, nn_e40_seed)."""
    z = ctypes.c_uint64()
    _native.check(_native.lib().nn_e40_seed(int(index), ctypes.byref(z)))
    return z.value


def e40_skip(state, k):
    z = ctypes.c_uint64()
    _native.check(_native.lib().nn_e40_skip(int(state), int(k) % (1 << 64), ctypes.byref(z)))
    return z.value


def e40_generate_into(state, out, stream=None, cfg=None):
    """The modulus-3^40 generator into the contiguous cuda tensor ``out``
    (uint64 or float64); returns the new state."""
    kind = _kind(out.dtype)
    if not out.is_cuda or not out.is_contiguous():
        raise NNError(_native.NN_EINVAL, "out must be a contiguous cuda tensor")
    st = ctypes.c_uint64(int(state))
    import torch
    with torch.cuda.device(out.device):
        rc = _native.lib().nn_e40_generate_ex(
            ctypes.byref(st), out.numel(), ctypes.c_void_p(out.data_ptr()), kind,
            _stream_handle(stream), ctypes.byref(cfg) if cfg is not None else None)
    _native.check(rc)
    return st.value


def e40_debug_mulmod(a, b, mulmod="montgomery"):
    """Host build of a 3^40 reduction ("montgomery" or "fp64", the limb
    step): a[i]*b[i] mod 3^40 (numpy uint64)."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    p = ctypes.POINTER(ctypes.c_uint64)
    _native.check(_native.lib().nn_e40_debug_mulmod_ex(
        MULMOD_NAMES[mulmod], a.ctypes.data_as(p), b.ctypes.data_as(p), a.size,
        out.ctypes.data_as(p)))
    return out


def dev_mult_pow(k):
    """(2^53)^k mod 3^33 in the device-side form (include/nn_device.h):
    (v, qh, ql) with qh + ql = v / 3^33 as a double-double."""
    m = _native.DevMult()
    _native.check(_native.lib().nn_dev_mult_pow(int(k), ctypes.byref(m)))
    return m.v, m.qh, m.ql


def dev_skip_table():
    """Device address (int) of the skip table nn_dev_skip reads, on the
    current device."""
    p = ctypes.c_void_p()
    _native.check(_native.lib().nn_dev_skip_table(ctypes.byref(p)))
    return p.value


def debug_mulmod(variant, a, b):
    """Host build of a step-loop reduction: a[i]*b[i] mod 3^33 (numpy uint64).
    ``variant``: a reduction name, or "device" for include/nn_device.h's
    nn_dev_mulmod."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    if isinstance(variant, str):
        variant = _native.NN_DEBUG_DEVICE_MULMOD if variant == "device" else MULMOD_NAMES[variant]
    p = ctypes.POINTER(ctypes.c_uint64)
    _native.check(_native.lib().nn_debug_mulmod(
        int(variant), a.ctypes.data_as(p), b.ctypes.data_as(p), a.size, out.ctypes.data_as(p)))
    return out


_DESC_DTYPE = [("state", "<u8"), ("length", "<u8"), ("out_offset", "<u8")]


def _batch_descs(states, lengths, out_offsets, out):
    import numpy as np
    n = len(states)
    descs = np.empty(n, dtype=_DESC_DTYPE)
    descs["state"] = np.asarray(states, dtype=np.uint64)
    descs["length"] = np.asarray(lengths, dtype=np.uint64)
    descs["out_offset"] = np.asarray(out_offsets, dtype=np.uint64)
    ends = descs["out_offset"] + descs["length"]
    if n and int(ends.max()) > out.numel():
        raise NNError(_native.NN_ERANGE, "a window ends past the output tensor")
    return descs


def generate_batch_static(states, lengths, out_offsets, out, stream=None, final_states=False):
    """nn_generate_batch_static: every stream's window written into the cuda
    tensor ``out`` (uint64 or float64) with no plan and no allocation (the
    library's static workspace).  Returns the final states as a numpy uint64
    array when ``final_states`` is true.  The descriptor array is kept
    alive until ``stream`` has passed the call (the copy is asynchronous)."""
    import numpy as np
    import torch
    if not out.is_cuda or not out.is_contiguous():
        raise NNError(_native.NN_EINVAL, "out must be a contiguous cuda tensor")
    kind = _kind(out.dtype)
    descs = _batch_descs(states, lengths, out_offsets, out)
    n = len(descs)
    fin = np.empty(n, dtype=np.uint64) if final_states else None
    p64 = ctypes.POINTER(ctypes.c_uint64)
    with torch.cuda.device(out.device):
        handle = _stream_handle(stream)
        rc = _native.lib().nn_generate_batch_static(
            ctypes.c_void_p(descs.ctypes.data), n, ctypes.c_void_p(out.data_ptr()), kind,
            handle, fin.ctypes.data_as(p64) if fin is not None else None)
        _native.check(rc)
        if n:
            # the host array must outlive the asynchronous copy that reads it
            s = torch.cuda.current_stream() if stream is None else stream
            s.synchronize()
    return fin


class BatchPlan:
    """A batch plan (include/nn.h, nn_batch_plan): many streams generated by
    one persistent kernel replayed from a hipGraph.

        plan = BatchPlan("f64", max_streams=10000, max_outputs=1 << 32)
        final = plan.generate(states, lengths, offsets, out)   # out: cuda tensor
    """

    def __init__(self, kind, max_streams, max_outputs, block=0, grid=0, mulmod=0,
                 temporal=False, graph=True, device=None, cluster=0, interleaved=False,
                 chunks=False, occupancy=0):
        import torch
        if isinstance(mulmod, str):
            mulmod = MULMOD_NAMES[mulmod]
        flags = (_native.NN_CFG_TEMPORAL_STORES if temporal else 0) | \
                (0 if graph else _native.NN_BATCH_NO_GRAPH) | \
                (_native.NN_BATCH_INTERLEAVED if interleaved else 0) | \
                (_native.NN_BATCH_CHUNKS if chunks else 0)
        cfg = _native.BatchCfg(int(block), int(grid), int(cluster), int(mulmod), flags,
                               int(occupancy))
        self.kind = _kind(kind)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else int(device))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _native.check(_native.lib().nn_batch_plan_create(
                self.kind, int(max_streams), int(max_outputs), ctypes.byref(cfg),
                ctypes.byref(handle)))
        self._h = handle

    def cfg(self):
        c = _native.BatchCfg()
        _native.check(_native.lib().nn_batch_plan_cfg(self._h, ctypes.byref(c)))
        return c

    def generate(self, states, lengths, out_offsets, out, stream=None, final_states=False):
        """Write every stream's window into the cuda tensor ``out`` (uint64 or
        float64, matching the plan's kind).  Returns the streams' final
        states as a numpy uint64 array when ``final_states`` is true."""
        import numpy as np
        import torch
        if self._h is None:
            raise NNError(_native.NN_EINVAL, "plan is closed")
        want = torch.uint64 if self.kind == NN_OUT_U64 else torch.float64
        if not out.is_cuda or not out.is_contiguous() or out.dtype != want:
            raise NNError(_native.NN_EINVAL, "out must be a contiguous cuda %s tensor" % want)
        n = len(states)
        descs = np.empty(n, dtype=_DESC_DTYPE)
        descs["state"] = np.asarray(states, dtype=np.uint64)
        descs["length"] = np.asarray(lengths, dtype=np.uint64)
        descs["out_offset"] = np.asarray(out_offsets, dtype=np.uint64)
        ends = descs["out_offset"] + descs["length"]
        if n and int(ends.max()) > out.numel():
            raise NNError(_native.NN_ERANGE, "a window ends past the output tensor")
        fin = np.empty(n, dtype=np.uint64) if final_states else None
        p64 = ctypes.POINTER(ctypes.c_uint64)
        with torch.cuda.device(out.device):
            rc = _native.lib().nn_generate_batch(
                self._h, ctypes.c_void_p(descs.ctypes.data), n, ctypes.c_void_p(out.data_ptr()),
                _stream_handle(stream), fin.ctypes.data_as(p64) if fin is not None else None)
        _native.check(rc)
        return fin

    def close(self):
        if getattr(self, "_h", None) is not None:
            _native.lib().nn_batch_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
