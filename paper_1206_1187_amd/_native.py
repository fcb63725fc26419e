"""ctypes loader for ``libnn.so`` (the C ABI declared in include/nn.h).

The library must have been built in-tree (``paper_1206_1187_amd/build.py``);
there is no fallback: a missing library raises ``NativeLibraryMissing``.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnn.so")

NN_OK, NN_EINVAL, NN_ERANGE, NN_EHIP, NN_ENOMEM, NN_ENODEV = range(6)
NN_OUT_U64, NN_OUT_F64 = 0, 1
(NN_MULMOD_DEFAULT, NN_MULMOD_FP64, NN_MULMOD_BARRETT, NN_MULMOD_SHOUP, NN_MULMOD_MONTGOMERY,
 NN_MULMOD_MODBARRETT) = range(6)
NN_CFG_TEMPORAL_STORES = 1
NN_CFG_ROWS = 2
NN_CFG_FLAT = 4
NN_CFG_CONSECUTIVE = 8
NN_CFG_PAPER_STRIDED = 16
NN_CFG_NONTEMPORAL_STORES = 32
NN_CFG_ADDRESS_ORDER = 128
NN_FILL_WITH_START = 64
NN_DEBUG_DEVICE_MULMOD = 100

MULMOD_NAMES = {
    "default": NN_MULMOD_DEFAULT,
    "fp64": NN_MULMOD_FP64,
    "barrett": NN_MULMOD_BARRETT,
    "shoup": NN_MULMOD_SHOUP,
    "montgomery": NN_MULMOD_MONTGOMERY,
    "modbarrett": NN_MULMOD_MODBARRETT,
}


class NativeLibraryMissing(RuntimeError):
    pass


class NNError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("nn status %d: %s" % (status, detail))


class LaunchCfg(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("mulmod", ctypes.c_uint32),
        ("unroll", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("occupancy", ctypes.c_uint32),
        ("ilp", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class StreamDesc(ctypes.Structure):
    """One stream of a batched call (see nn_stream_desc in include/nn.h)."""
    _fields_ = [
        ("state", ctypes.c_uint64),
        ("length", ctypes.c_uint64),
        ("out_offset", ctypes.c_uint64),
    ]


class BatchCfg(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("cluster", ctypes.c_uint32),
        ("mulmod", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("occupancy", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


NN_BATCH_NO_GRAPH = 8
NN_BATCH_INTERLEAVED = 16
NN_BATCH_CHUNKS = 32


_u64 = ctypes.c_uint64
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p
_int = ctypes.c_int

NN_SERVER_FAKE_DEVICE = 1
NN_SERVER_DEVICE_QUEUE = 2
NN_ECANCELED = 6


class ServerCfg(ctypes.Structure):
    _fields_ = [
        ("pool", ctypes.c_void_p),
        ("pool_bytes", ctypes.c_uint64),
        ("max_batch_outputs", ctypes.c_uint64),
        ("max_batch_requests", ctypes.c_uint32),
        ("max_slots", ctypes.c_uint32),
        ("lanes", ctypes.c_uint32),
        ("kind", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("batch", BatchCfg),
        ("fake_latency_s", ctypes.c_double),
        ("fake_bytes_per_s", ctypes.c_double),
        ("queue_max_outputs", ctypes.c_uint64),
        ("queue_workgroups", ctypes.c_uint32),
        ("queue_capacity", ctypes.c_uint32),
        ("queue_idle_s", ctypes.c_double),
    ]


class Completion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("count", ctypes.c_uint64),
        ("position", ctypes.c_uint64),
        ("data", ctypes.c_void_p),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_launch", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("stream_id", ctypes.c_uint32),
        ("status", ctypes.c_int32),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "failed", "released", "in_flight", "batches", "queued",
        "pending", "pool_used", "pool_peak", "slots_used")] + [("now", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}



# name -> (restype, argtypes); must match include/nn.h
class DevMult(ctypes.Structure):
    """nn_dev_mult (include/nn.h): a multiplier for the device-side API."""
    _fields_ = [("v", ctypes.c_double), ("qh", ctypes.c_double), ("ql", ctypes.c_double)]


SIGNATURES = {
    "nn_seed": (_int, [_u64, _pu64]),
    "nn_skip": (_int, [_u64, _u64, _pu64]),
    "nn_init": (_int, [_int]),
    "nn_generate": (_int, [_pu64, _u64, _vp, _int, _vp]),
    "nn_generate_ex": (_int, [_pu64, _u64, _vp, _int, _vp, ctypes.POINTER(LaunchCfg)]),
    "nn_default_cfg": (_int, [_int, _u64, ctypes.POINTER(LaunchCfg)]),
    "nn_fill": (_int, [_u64, _vp, _u64, _vp, ctypes.POINTER(LaunchCfg)]),
    "nn_consume": (_int, [_pu64, _u64, _int, _vp, _vp, ctypes.POINTER(LaunchCfg)]),
    "nn_dev_mult_pow": (_int, [_u64, ctypes.POINTER(DevMult)]),
    "nn_e40_seed": (_int, [_u64, _pu64]),
    "nn_e40_skip": (_int, [_u64, _u64, _pu64]),
    "nn_e40_generate": (_int, [_pu64, _u64, _vp, _int, _vp]),
    "nn_e40_generate_ex": (_int, [_pu64, _u64, _vp, _int, _vp, ctypes.POINTER(LaunchCfg)]),
    "nn_e40_debug_mulmod": (_int, [_pu64, _pu64, _u64, _pu64]),
    "nn_e40_debug_mulmod_ex": (_int, [_int, _pu64, _pu64, _u64, _pu64]),
    "nn_dev_skip_table": (_int, [ctypes.POINTER(ctypes.c_void_p)]),
    "nn_strerror": (ctypes.c_char_p, [_int]),
    "nn_last_error": (ctypes.c_char_p, []),
    "nn_version": (ctypes.c_char_p, []),
    "nn_debug_mulmod": (_int, [_int, _pu64, _pu64, _u64, _pu64]),
    "nn_batch_plan_create": (_int, [_int, ctypes.c_uint32, _u64, ctypes.POINTER(BatchCfg),
                                    ctypes.POINTER(_vp)]),
    "nn_batch_plan_destroy": (_int, [_vp]),
    "nn_batch_plan_cfg": (_int, [_vp, ctypes.POINTER(BatchCfg)]),
    "nn_generate_batch": (_int, [_vp, _vp, ctypes.c_uint32, _vp, _vp, _pu64]),
    "nn_generate_batch_static": (_int, [_vp, ctypes.c_uint32, _vp, _int, _vp, _pu64]),
}

_SERVER_SIGNATURES = {
    "nn_server_create": (ctypes.c_int, [ctypes.POINTER(ServerCfg), ctypes.c_void_p,
                                        ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "nn_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nn_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "nn_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Completion),
                                      ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "nn_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "nn_server_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "nn_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "nn_server_set_clock": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "nn_server_inject_failures": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
}




class ReplayStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("requests", ctypes.c_uint64),
                ("variates", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("seen_p50", ctypes.c_double), ("seen_p99", ctypes.c_double),
                ("launch_p50", ctypes.c_double), ("launch_p99", ctypes.c_double),
                ("done_p50", ctypes.c_double), ("done_p99", ctypes.c_double)]


_pd = ctypes.POINTER(ctypes.c_double)
_SERVER_SIGNATURES.update({
    "nn_server_replay": (ctypes.c_int, [ctypes.c_void_p, _pd, ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64,
                                        ctypes.c_double, ctypes.c_double, _pd,
                                        ctypes.POINTER(ReplayStats)]),
    "nn_replay_per_request": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32, _pd,
                                             ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                             ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, _pd,
                                             ctypes.POINTER(ReplayStats)]),
})
SIGNATURES.update(_SERVER_SIGNATURES)

_lib = None


def lib():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryMissing(
                "%s is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
                "or `python paper_1206_1187_amd/build.py`" % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(handle, name):
                fn = getattr(handle, name)
                fn.restype = res
                fn.argtypes = args
        _lib = handle
    return _lib


def check(status):
    if status != NN_OK:
        detail = lib().nn_last_error().decode() or lib().nn_strerror(status).decode()
        raise NNError(status, detail)
    return status
