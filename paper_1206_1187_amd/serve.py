"""The served form (include/nn.h, nn_server_*): binding and trace replay.

``Server`` wraps the C++ scheduler: requests (stream, count) are queued,
admitted from the head of the queue while the output pool has room, and
launched as batches on several HIP streams.  ``replay_served`` drives a
timestamped arrival trace through a server in real time and reports
latency percentiles and throughput; ``replay_plain`` serves the same trace
with one nn_generate launch per request, for comparison.
"""
import ctypes
import time

import numpy as np

from . import _native
from ._native import (NN_ECANCELED, NN_OUT_F64, NN_OUT_U64, NN_SERVER_FAKE_DEVICE,  # noqa: F401
                      BatchCfg, Completion, NNError, ServerCfg, ServerStats)


def _lib():
    return _native.lib()


class Server:
    """A continuous-batching server over ``stream_states`` (one state per
    client stream at position 0).

    On a GPU the output pool is a torch tensor owned by this object and
    completions carry views into it; with ``fake=True`` the scheduler runs
    on the host (simulated clock, exact host arithmetic) for testing."""

    def __init__(self, stream_states, pool_bytes, kind="f64", lanes=2, max_batch_outputs=0,
                 max_batch_requests=0, max_slots=0, fake=False, fake_latency_s=0.0,
                 fake_bytes_per_s=0.0, device_queue=False, queue_max_outputs=0,
                 queue_workgroups=0, queue_capacity=0, queue_idle_s=0.0, **batch_kw):
        from . import MULMOD_NAMES
        kind = NN_OUT_U64 if kind in ("u64", NN_OUT_U64) else NN_OUT_F64
        self.kind = kind
        self.fake = bool(fake)
        mulmod = batch_kw.get("mulmod", 0)
        if isinstance(mulmod, str):
            mulmod = MULMOD_NAMES[mulmod]
        batch = BatchCfg(int(batch_kw.get("block", 0)), int(batch_kw.get("grid", 0)),
                         int(batch_kw.get("cluster", 0)), int(mulmod),
                         (_native.NN_CFG_TEMPORAL_STORES if batch_kw.get("temporal") else 0) |
                         (_native.NN_BATCH_INTERLEAVED if batch_kw.get("interleaved") else 0) |
                         (_native.NN_BATCH_CHUNKS if batch_kw.get("chunks") else 0),
                         int(batch_kw.get("occupancy", 0)))
        self.pool_bytes = int(pool_bytes) & ~255
        self.pool = None
        pool_ptr = None
        if not self.fake:
            import torch
            self.pool = torch.empty(self.pool_bytes // 8, dtype=torch.int64, device="cuda")
            pool_ptr = self.pool.data_ptr()
        flags = (NN_SERVER_FAKE_DEVICE if self.fake else 0) | \
            (_native.NN_SERVER_DEVICE_QUEUE if device_queue else 0)
        cfg = ServerCfg(pool_ptr, self.pool_bytes, int(max_batch_outputs),
                        int(max_batch_requests), int(max_slots), int(lanes), kind, flags, batch,
                        float(fake_latency_s), float(fake_bytes_per_s), int(queue_max_outputs),
                        int(queue_workgroups), int(queue_capacity), float(queue_idle_s))
        st = np.ascontiguousarray(stream_states, dtype=np.uint64)
        h = ctypes.c_void_p()
        _native.check(_lib().nn_server_create(ctypes.byref(cfg), st.ctypes.data, st.size,
                                               ctypes.byref(h)))
        self._h = h
        self._buf = (Completion * 4096)()

    def submit(self, stream_id, count):
        t = ctypes.c_uint64()
        _native.check(_lib().nn_server_submit(self._h, int(stream_id), int(count),
                                              ctypes.byref(t)))
        return int(t.value)

    def poll(self):
        """Progress, then the finished requests (list of Completion copies)."""
        out = []
        n = ctypes.c_uint32()
        while True:
            _native.check(_lib().nn_server_poll(self._h, self._buf, len(self._buf),
                                                ctypes.byref(n)))
            out.extend(Completion.from_buffer_copy(self._buf[i]) for i in range(n.value))
            if n.value < len(self._buf):
                return out

    def release(self, ticket):
        _native.check(_lib().nn_server_release(self._h, int(ticket)))

    def cancel(self, ticket):
        _native.check(_lib().nn_server_cancel(self._h, int(ticket)))

    def stats(self):
        s = ServerStats()
        _native.check(_lib().nn_server_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()

    def set_clock(self, now):
        _native.check(_lib().nn_server_set_clock(self._h, float(now)))

    def inject_failures(self, n):
        _native.check(_lib().nn_server_inject_failures(self._h, int(n)))

    def data(self, c):
        """The outputs of a completion: a torch view into the pool (GPU) or a
        numpy copy (fake device), as uint64 bit patterns."""
        if c.count == 0 or not c.data:
            return np.empty(0, dtype=np.uint64)
        if self.fake:
            return np.frombuffer(ctypes.string_at(c.data, 8 * c.count), dtype=np.uint64).copy()
        off = (c.data - self.pool.data_ptr()) // 8
        return self.pool[off:off + c.count]

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib().nn_server_destroy(self._h)
            self._h = None
        self.pool = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _percentiles(lat):
    if not len(lat):
        return {}
    a = np.asarray(lat)
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "max_ms": float(a.max() * 1e3), "mean_ms": float(a.mean() * 1e3)}


def replay_served(server, trace, time_scale=1.0, consumer=None, timeout_s=None):
    """Drive ``trace`` (workloads.ServedTrace) through ``server`` in real time
    (arrival times divided by ``time_scale``).  Each completion is handed to
    ``consumer(server, completion)`` (if given) and then released.  Returns
    latency percentiles (completion observed minus arrival) and throughput."""
    t_arr = np.asarray(trace.t_arrive) / float(time_scale)
    sid = np.asarray(trace.stream_id)
    cnt = np.asarray(trace.count)
    n = len(t_arr)
    arrival = {}
    lat = []
    failed = 0
    done = 0
    i = 0
    clock0 = server.stats()["now"]
    t0 = time.perf_counter()
    deadline = None if timeout_s is None else t0 + timeout_s
    while done < n:
        now = time.perf_counter() - t0
        while i < n and t_arr[i] <= now:
            arrival[server.submit(int(sid[i]), int(cnt[i]))] = t_arr[i]
            i += 1
        for c in server.poll():
            lat.append((c.t_done - clock0) - arrival.pop(c.ticket))
            if c.status != 0:
                failed += 1
            elif consumer is not None:
                consumer(server, c)
            server.release(c.ticket)
            done += 1
        if deadline is not None and time.perf_counter() > deadline:
            raise TimeoutError("served replay did not finish: %d of %d done" % (done, n))
    wall = time.perf_counter() - t0
    total = int(cnt.sum())
    res = {"requests": n, "variates": total, "wall_s": wall, "variates_per_s": total / wall,
           "failed": failed, "stats": server.stats()}
    res.update(_percentiles(lat))
    return res


def replay_plain(trace, stream_states, pool_elems, kind="f64", time_scale=1.0, timeout_s=None):
    """The same trace with one nn_generate launch per request on one HIP
    stream, outputs in a ring over a pool of ``pool_elems`` outputs (a
    request waits for space as the oldest finish).  Window positions follow
    arrival order per stream, as in the server."""
    import torch

    import paper_1206_1187_amd as nn
    P = nn.PERIOD
    dt = torch.float64 if kind == "f64" else torch.uint64
    pool = torch.empty(int(pool_elems), dtype=dt, device="cuda")
    t_arr = np.asarray(trace.t_arrive) / float(time_scale)
    sid = np.asarray(trace.stream_id)
    cnt = np.asarray(trace.count)
    states = [int(s) for s in stream_states]
    pos = [0] * len(states)
    n = len(t_arr)
    inflight = []  # (event, arrival, start, count) in launch order
    head = 0       # next free element of the ring
    used = 0
    lat = []
    i = 0
    done = 0
    t0 = time.perf_counter()
    deadline = None if timeout_s is None else t0 + timeout_s
    while done < n:
        now = time.perf_counter() - t0
        while i < n and t_arr[i] <= now:
            c = int(cnt[i])
            start = head if head + c <= pool.numel() else 0
            waste = pool.numel() - head if start == 0 and head != 0 else 0
            if used + waste + c > pool.numel():
                break  # wait for the oldest to finish
            s = int(sid[i])
            st = nn.skip(states[s], pos[s])
            pos[s] = (pos[s] + c) % P
            nn.generate_into(st, pool[start:start + c])
            ev = torch.cuda.Event()
            ev.record()
            inflight.append((ev, t_arr[i], start, c, waste))
            used += waste + c
            head = start + c
            i += 1
        while inflight and inflight[0][0].query():
            ev, ta, start, c, waste = inflight.pop(0)
            lat.append(time.perf_counter() - t0 - ta)
            used -= waste + c
            done += 1
        if deadline is not None and time.perf_counter() > deadline:
            raise TimeoutError("plain replay did not finish: %d of %d done" % (done, n))
    wall = time.perf_counter() - t0
    total = int(cnt.sum())
    res = {"requests": n, "variates": total, "wall_s": wall, "variates_per_s": total / wall}
    res.update(_percentiles(lat))
    return res


def _trace_arrays(trace, n=None):
    t = np.ascontiguousarray(trace.t_arrive[:n], dtype=np.float64)
    s = np.ascontiguousarray(trace.stream_id[:n], dtype=np.uint32)
    c = np.ascontiguousarray(trace.count[:n], dtype=np.uint64)
    return t, s, c


#: Results split latency at requests of this many outputs (the median
#: request size of the served workload is about 2^16).
SMALL_REQUEST = 1 << 16


def _result(lat, st, count=None):
    res = {"requests": int(st.requests), "variates": int(st.variates), "wall_s": st.wall_s,
           "variates_per_s": st.variates / st.wall_s if st.wall_s > 0 else 0.0,
           "failed": int(st.failed)}
    res.update(_percentiles(lat))
    if count is not None:
        small = np.asarray(count) <= SMALL_REQUEST
        for name, sel in (("small", small), ("large", ~small)):
            pc = _percentiles(np.asarray(lat)[sel])
            res["%s_p50_ms" % name] = pc.get("p50_ms", 0.0)
            res["%s_p99_ms" % name] = pc.get("p99_ms", 0.0)
    res["stages_ms"] = {k: getattr(st, k) * 1e3 for k in
                        ("seen_p50", "seen_p99", "launch_p50", "launch_p99", "done_p50",
                         "done_p99")}
    return res


def replay_served_native(server, trace, time_scale=1.0, timeout_s=0.0, n=None):
    """``replay_served`` with the arrival loop in the library (no Python in
    the loop); outputs are released as soon as they are reported."""
    t, s, c = _trace_arrays(trace, n)
    lat = np.zeros(t.size, dtype=np.float64)
    st = _native.ReplayStats()
    pd = ctypes.POINTER(ctypes.c_double)
    _native.check(_lib().nn_server_replay(
        server._h, t.ctypes.data_as(pd), s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
        c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), t.size, float(time_scale),
        float(timeout_s), lat.ctypes.data_as(pd), ctypes.byref(st)))
    return _result(lat, st, c)


def replay_per_request_native(trace, stream_states, pool_elems, kind="f64", time_scale=1.0,
                              timeout_s=0.0, n=None):
    """One nn_generate launch per request on torch's current stream, with the
    arrival loop in the library."""
    import torch
    t, s, c = _trace_arrays(trace, n)
    states = np.ascontiguousarray(stream_states, dtype=np.uint64)
    pool = torch.empty(int(pool_elems), dtype=torch.float64 if kind == "f64" else torch.uint64,
                       device="cuda")
    lat = np.zeros(t.size, dtype=np.float64)
    st = _native.ReplayStats()
    pd = ctypes.POINTER(ctypes.c_double)
    p64 = ctypes.POINTER(ctypes.c_uint64)
    _native.check(_lib().nn_replay_per_request(
        states.ctypes.data_as(p64), states.size, t.ctypes.data_as(pd),
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), c.ctypes.data_as(p64), t.size,
        float(time_scale), float(timeout_s), ctypes.c_void_p(pool.data_ptr()), pool.numel(),
        NN_OUT_F64 if kind == "f64" else NN_OUT_U64,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), lat.ctypes.data_as(pd),
        ctypes.byref(st)))
    del pool
    return _result(lat, st, c)
