"""GPU tests of the served form: every served request equals the oracle on
its window and equals the plain path run alone on the same window."""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402
from paper_1206_1187_amd import serve  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _states(n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(wl.INDEX_MIN, wl.INDEX_MAX, n, endpoint=True, dtype=np.int64)
    return np.array([orc.seed(int(a)) for a in idx], dtype=np.uint64)


def _bits(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    nn.init(0)
    yield
    torch.cuda.synchronize()


LANE_SHAPES = {"blocked": {}, "interleaved": dict(interleaved=True, block=128),
               "chunked": dict(chunks=True, temporal=True)}


@pytest.mark.parametrize("kind,shape", [("f64", "blocked"), ("u64", "blocked"),
                                        ("f64", "interleaved"), ("u64", "interleaved"),
                                        ("f64", "chunked"), ("u64", "chunked")])
def test_served_requests_equal_oracle_and_plain_alone(kind, shape):
    """Every batch kernel in the server's indexed mode (states read from the
    device table; the chunked kernel with its windows sorted by pool offset,
    one workgroup per chunk)."""
    _say("served", kind, shape)
    states = _states(8, 21)
    rng = np.random.default_rng(22)
    reqs = [(int(rng.integers(0, 8)), int(np.floor(np.exp(rng.uniform(0, np.log(1 << 18))))))
            for _ in range(300)] + [(3, 0), (5, 1), (5, (1 << 20) + 3)]
    with serve.Server(states, 1 << 28, kind=kind, lanes=3, max_batch_requests=32,
                      **LANE_SHAPES[shape]) as srv:
        tickets = [srv.submit(s, n) for s, n in reqs]
        done = {}
        while len(done) < len(reqs):
            for c in srv.poll():
                done[c.ticket] = c
        pos = [0] * 8
        for t, (s, n) in zip(tickets, reqs):
            c = done[t]
            assert c.status == 0 and c.position == pos[s]
            pos[s] += n
            got = _bits(srv.data(c)) if n else np.empty(0, dtype=np.uint64)
            ref, _ = orc.gen(orc.skip(int(states[s]), c.position), n, kind)
            assert np.array_equal(got, ref.view(np.uint64)), (t, s, n)
            if 0 < n <= 1 << 16:  # alone: the plain path on the same window
                alone, _ = nn.generate(nn.skip(int(states[s]), c.position), n, kind)
                torch.cuda.synchronize()
                assert np.array_equal(_bits(alone), got)
            srv.release(t)
        st = srv.stats()
        assert st["pool_used"] == 0 and st["released"] == len(reqs) and st["batches"] >= 10


def _full_check(states, bad):
    """A replay consumer comparing all of a completed f64 request's outputs
    with the oracle on its window (its stream's state skipped to the
    window's position); failing tickets go to `bad`."""
    buf = np.empty(1 << 24, dtype=np.float64)

    def consumer(server, c):
        ref = buf[:c.count]
        orc.gen_into(orc.skip(int(states[c.stream_id]), c.position), ref, threads=0)
        if not np.array_equal(_bits(server.data(c)), ref.view(np.uint64)):
            bad.append(c.ticket)
    return consumer


def test_served_trace_slice_checked_per_request():
    """A slice of the served workload (Poisson arrivals, sizes log-uniform in
    [256, 2^24]) replayed in real time; every output of every request is
    checked against the oracle before release."""
    tr = wl.served()
    n = 600
    sl = wl.ServedTrace(tr.stream_indices, tr.t_arrive[:n], tr.stream_id[:n], tr.count[:n])
    states = np.array([orc.seed(int(a)) for a in tr.stream_indices], dtype=np.uint64)
    bad = []
    consumer = _full_check(states, bad)

    with serve.Server(states, 16 << 30, lanes=2) as srv:
        res = serve.replay_served(srv, sl, consumer=consumer, timeout_s=60)
    _say("served slice", res)
    assert not bad and res["failed"] == 0 and res["requests"] == n


def test_pool_pressure_admission_and_cancel_on_device():
    """A pool far smaller than the demand: requests wait at the head of the
    queue until releases free memory, a queued request cancelled meanwhile
    completes with NN_ECANCELED and keeps its window, and every served
    request equals the oracle on its whole window."""
    states = _states(4, 31)
    pool_bytes = 8 << 20  # 1 Mi f64
    rng = np.random.default_rng(32)
    reqs = [(int(rng.integers(0, 4)), int(rng.integers(1, 300_000))) for _ in range(80)]
    with serve.Server(states, pool_bytes, lanes=2) as srv:
        tickets = [srv.submit(s, n) for s, n in reqs]
        victim = tickets[-1]
        srv.cancel(victim)
        done = {}
        guard = 0
        while len(done) < len(reqs):
            for c in srv.poll():
                done[c.ticket] = c
                if c.ticket == victim:
                    assert c.status == serve.NN_ECANCELED
                    continue
                assert c.status == 0
                ref, _ = orc.gen(orc.skip(int(states[c.stream_id]), c.position), c.count, "f64")
                assert np.array_equal(_bits(srv.data(c)), ref.view(np.uint64))
                srv.release(c.ticket)
            guard += 1
            assert guard < 10_000_000
        srv.release(victim)
        pos = [0] * 4
        for t, (s, n) in zip(tickets, reqs):
            assert done[t].position == pos[s]  # windows fixed at submission
            pos[s] += n
        st = srv.stats()
        assert st["pool_used"] == 0 and st["pool_peak"] <= pool_bytes


def test_destroy_with_batches_in_flight():
    """Closing a server while its batches run waits for them; a new server
    on the same device then works."""
    states = _states(2, 41)
    srv = serve.Server(states, 1 << 30, lanes=2)
    for _ in range(20):
        srv.submit(0, 1 << 22)
    srv.poll()  # admits and launches
    srv.close()
    torch.cuda.synchronize()
    with serve.Server(states, 1 << 24, lanes=1) as srv2:
        t = srv2.submit(1, 1000)
        got = []
        while not got:
            got = srv2.poll()
        ref, _ = orc.gen(int(states[1]), 1000, "f64")
        assert got[0].ticket == t and np.array_equal(_bits(srv2.data(got[0])), ref.view(np.uint64))
        srv2.release(t)


def _drain(srv, n, limit=5_000_000):
    done = {}
    k = 0
    while len(done) < n:
        for c in srv.poll():
            done[c.ticket] = c
        k += 1
        assert k < limit, "server did not finish"
    return done


@pytest.mark.parametrize("kind", ["f64", "u64"])
def test_device_queue_requests_equal_oracle(kind):
    """Requests served by the persistent device queue (no launch per
    request) and, above its size limit or with its ring full, by the batch
    lanes: every request equals the oracle on its window and the plain path
    run alone."""
    states = _states(8, 51)
    rng = np.random.default_rng(52)
    sizes = [1, 2, 3, 511, 512, 513, 1023, 1024, 1025, 65_535, 65_536, 65_537, 300_000]
    reqs = [(int(rng.integers(0, 8)), s) for s in sizes]
    reqs += [(int(rng.integers(0, 8)), int(np.floor(np.exp(rng.uniform(0, np.log(1 << 17))))))
             for _ in range(400)]
    with serve.Server(states, 1 << 28, kind=kind, lanes=2, device_queue=True,
                      queue_max_outputs=1 << 16, queue_capacity=64) as srv:
        tickets = [srv.submit(s, n) for s, n in reqs]
        done = _drain(srv, len(reqs))
        pos = [0] * 8
        for t, (s, n) in zip(tickets, reqs):
            c = done[t]
            assert c.status == 0 and c.position == pos[s]
            pos[s] += n
            got = _bits(srv.data(c))
            ref, _ = orc.gen(orc.skip(int(states[s]), c.position), n, kind)
            assert np.array_equal(got, ref.view(np.uint64)), (t, s, n)
            if n <= 1 << 12:
                alone, _ = nn.generate(nn.skip(int(states[s]), c.position), n, kind)
                torch.cuda.synchronize()
                assert np.array_equal(_bits(alone), got)
            srv.release(t)
        assert srv.stats()["pool_used"] == 0


def test_device_queue_idle_exit_and_relaunch():
    """The queue kernel leaves after a short idle time and is relaunched on
    the next request, which is served correctly."""
    import time
    states = _states(2, 61)
    with serve.Server(states, 1 << 24, lanes=1, device_queue=True, queue_idle_s=0.002) as srv:
        pos = 0
        for rep in range(4):
            t = srv.submit(1, 5000 + rep)
            c = _drain(srv, 1)[t]
            ref, _ = orc.gen(orc.skip(int(states[1]), pos), 5000 + rep, "f64")
            assert c.position == pos and np.array_equal(_bits(srv.data(c)), ref.view(np.uint64))
            pos += 5000 + rep
            srv.release(t)
            time.sleep(0.03)  # the kernel leaves meanwhile


def test_device_queue_trace_slice():
    """A slice of the served workload with the device queue: every output of
    every request against the oracle."""
    tr = wl.served()
    n = 600
    sl = wl.ServedTrace(tr.stream_indices, tr.t_arrive[:n], tr.stream_id[:n], tr.count[:n])
    states = np.array([orc.seed(int(a)) for a in tr.stream_indices], dtype=np.uint64)
    bad = []
    consumer = _full_check(states, bad)

    with serve.Server(states, 16 << 30, lanes=2, device_queue=True) as srv:
        res = serve.replay_served(srv, sl, consumer=consumer, timeout_s=60)
    _say("device queue slice", res)
    assert not bad and res["failed"] == 0 and res["requests"] == n


def test_device_queue_config_validation():
    states = _states(2, 71)
    for kw in (dict(queue_capacity=1000), dict(queue_capacity=1 << 21), dict(queue_workgroups=2000),
               dict(queue_idle_s=30.0)):
        with pytest.raises(nn.NNError):
            serve.Server(states, 1 << 20, device_queue=True, **kw)
