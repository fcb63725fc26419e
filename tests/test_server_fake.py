"""CPU tests of the served form's scheduler on the fake device (host pool,
simulated clock, exact host arithmetic): admission by pool bytes and
slots, head-of-line order, windows fixed at submission, batching limits,
out-of-order lane completion, injected launch failures and cancellation.
Expected outputs come from the oracle."""
import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import serve
from paper_1206_1187_amd import workloads as wl

M = 3 ** 33
P = 2 * 3 ** 32


def _states(n, seed=0):
    rng = np.random.default_rng(seed)
    idx = rng.integers(wl.INDEX_MIN, wl.INDEX_MAX, n, endpoint=True, dtype=np.int64)
    return np.array([orc.seed(int(a)) for a in idx], dtype=np.uint64)


def _expect(states, c, kind):
    ref, _ = orc.gen(orc.skip(int(states[c.stream_id]), c.position), c.count, kind)
    return ref.view(np.uint64)


def _drain(srv, clock=None):
    out = []
    for _ in range(1000):
        if clock is not None:
            clock[0] += 1.0
            srv.set_clock(clock[0])
        got = srv.poll()
        out.extend(got)
        st = srv.stats()
        if not got and st["queued"] == 0 and st["in_flight"] == 0 and st["pending"] == 0:
            break
    return out


@pytest.mark.parametrize("kind", ["u64", "f64"])
def test_outputs_and_windows_follow_arrival_order(kind):
    states = _states(5, 1)
    rng = np.random.default_rng(2)
    with serve.Server(states, 1 << 22, kind=kind, fake=True, lanes=2) as srv:
        subs = []
        for _ in range(60):
            s = int(rng.integers(0, 5))
            n = int(rng.integers(0, 3000))
            subs.append((srv.submit(s, n), s, n))
        comps = {c.ticket: c for c in _drain(srv, [0.0])}
        assert len(comps) == len(subs)
        pos = [0] * 5
        for t, s, n in subs:
            c = comps[t]
            assert c.status == 0 and c.stream_id == s and c.count == n
            assert c.position == pos[s]  # windows in arrival order per stream
            pos[s] += n
            assert np.array_equal(srv.data(c), _expect(states, c, kind))
            srv.release(t)
        st = srv.stats()
        assert st["pool_used"] == 0 and st["slots_used"] == 0 and st["released"] == 60


def test_pool_exhaustion_blocks_head_of_line_until_release():
    states = _states(2, 3)
    pool = 64 * 1024  # 8192 outputs
    with serve.Server(states, pool, fake=True, lanes=4) as srv:
        a = srv.submit(0, 5000)
        b = srv.submit(1, 5000)   # does not fit next to a
        c = srv.submit(0, 10)     # small, but queued behind b (head of line)
        srv.set_clock(1.0)
        got = srv.poll()
        assert [x.ticket for x in got] == [a]
        st = srv.stats()
        assert st["queued"] == 2 and st["pool_used"] == 5000 * 8 + (256 - 5000 * 8 % 256) % 256
        srv.set_clock(2.0)
        assert srv.poll() == []          # nothing freed yet
        srv.release(a)
        srv.set_clock(3.0)
        got = srv.poll()
        assert sorted(x.ticket for x in got) == [b, c]
        for x in got:
            assert np.array_equal(srv.data(x), _expect(states, x, "f64"))
            srv.release(x.ticket)


def test_request_larger_than_pool_or_batch_is_refused():
    states = _states(1, 4)
    with serve.Server(states, 4096, fake=True, max_batch_outputs=300) as srv:
        with pytest.raises(serve.NNError):
            srv.submit(0, 513)   # 4104 bytes > pool
        with pytest.raises(serve.NNError):
            srv.submit(0, 301)   # > max_batch_outputs
        with pytest.raises(serve.NNError):
            srv.submit(1, 10)    # unknown stream
        t = srv.submit(0, 300)
        got = _drain(srv, [0.0])
        assert [x.ticket for x in got] == [t] and got[0].position == 0


def test_burst_is_split_into_bounded_batches():
    states = _states(3, 5)
    with serve.Server(states, 1 << 24, fake=True, lanes=1, max_batch_requests=16,
                      max_batch_outputs=4000) as srv:
        ts = [srv.submit(i % 3, 100 + i) for i in range(200)]
        comps = _drain(srv, [0.0])
        assert sorted(c.ticket for c in comps) == ts
        st = srv.stats()
        # at most 16 requests and 4000 outputs per batch
        assert st["batches"] >= max(200 // 16, sum(100 + i for i in range(200)) // 4000)
        for c in comps:
            assert np.array_equal(srv.data(c), _expect(states, c, "f64"))
            srv.release(c.ticket)


def test_out_of_order_lane_completion():
    """A long batch on one lane, short ones on another: completions come back
    in completion order, each with its own data."""
    states = _states(2, 6)
    with serve.Server(states, 1 << 22, fake=True, lanes=2, fake_latency_s=1.0,
                      fake_bytes_per_s=8e4) as srv:
        big = srv.submit(0, 40_000)      # 320 KB -> 5 s on the model
        srv.set_clock(0.5)
        assert srv.poll() == []
        small = srv.submit(1, 100)       # second lane, 1.01 s
        srv.set_clock(0.6)
        srv.poll()
        srv.set_clock(2.0)
        got = srv.poll()
        assert [c.ticket for c in got] == [small]
        srv.set_clock(10.0)
        got2 = srv.poll()
        assert [c.ticket for c in got2] == [big]
        for c in got + got2:
            assert c.t_done >= c.t_launch >= c.t_admit >= c.t_submit
            assert np.array_equal(srv.data(c), _expect(states, c, "f64"))
            srv.release(c.ticket)


def test_injected_launch_failure_frees_and_keeps_windows():
    states = _states(2, 7)
    with serve.Server(states, 1 << 20, fake=True, lanes=1, max_batch_requests=2) as srv:
        srv.inject_failures(1)
        t1 = srv.submit(0, 50)
        t2 = srv.submit(0, 60)
        t3 = srv.submit(0, 70)
        comps = {c.ticket: c for c in _drain(srv, [0.0])}
        assert comps[t1].status == 3 and comps[t2].status == 3  # NN_EHIP
        assert comps[t3].status == 0
        # the failed windows stay assigned: the next request starts at 110
        assert comps[t3].position == 110
        assert np.array_equal(srv.data(comps[t3]), _expect(states, comps[t3], "f64"))
        for t in (t1, t2, t3):
            srv.release(t)
        assert srv.stats()["pool_used"] == 0 and srv.stats()["failed"] == 2


def test_cancel_queued_request():
    states = _states(1, 8)
    with serve.Server(states, 8192, fake=True, lanes=1) as srv:
        a = srv.submit(0, 1000)   # fills the pool
        b = srv.submit(0, 10)
        c = srv.submit(0, 20)
        srv.set_clock(0.1)
        srv.poll()
        srv.cancel(b)
        with pytest.raises(serve.NNError):
            srv.cancel(a)         # already admitted
        got = {x.ticket: x for x in srv.poll()}
        assert got[b].status == serve.NN_ECANCELED
        srv.release(b)
        srv.release(a)
        rest = {x.ticket: x for x in _drain(srv, [1.0])}
        assert rest[c].position == 1010  # b's window stays assigned
        assert np.array_equal(srv.data(rest[c]), _expect(states, rest[c], "f64"))


def test_slot_limit():
    states = _states(1, 9)
    with serve.Server(states, 1 << 20, fake=True, max_slots=3) as srv:
        ts = [srv.submit(0, 10) for _ in range(5)]
        srv.set_clock(1.0)
        first = srv.poll()
        assert len(first) == 3 and srv.stats()["queued"] == 2
        for c in first:
            srv.release(c.ticket)
        rest = _drain(srv, [2.0])
        assert sorted(c.ticket for c in first + rest) == ts


def test_release_rules():
    states = _states(1, 10)
    with serve.Server(states, 1 << 16, fake=True) as srv:
        t = srv.submit(0, 10)
        with pytest.raises(serve.NNError):
            srv.release(t)        # not finished
        with pytest.raises(serve.NNError):
            srv.release(999)      # unknown
        got = _drain(srv, [0.0])
        srv.release(got[0].ticket)
        with pytest.raises(serve.NNError):
            srv.release(t)        # twice


def test_same_result_alone_and_in_the_mix():
    """A request's bytes depend only on (stream, window): served alone in a
    fresh server (after the same earlier windows of its stream) or amid
    other traffic, they are identical."""
    states = _states(4, 11)
    rng = np.random.default_rng(12)
    plan = [(int(rng.integers(0, 4)), int(rng.integers(1, 2000))) for _ in range(40)]
    with serve.Server(states, 1 << 22, fake=True, lanes=3, max_batch_requests=5) as mix:
        tickets = [mix.submit(s, n) for s, n in plan]
        mixed = {c.ticket: (c, mix.data(c)) for c in _drain(mix, [0.0])}
    for k in (0, 7, 19, 39):
        s, n = plan[k]
        with serve.Server(states, 1 << 22, fake=True, lanes=1) as alone:
            # the same earlier windows of stream s, then the request itself
            for s2, n2 in plan[:k]:
                if s2 == s:
                    alone.submit(s2, n2)
            t = alone.submit(s, n)
            got = {c.ticket: c for c in _drain(alone, [0.0])}
            c, d = mixed[tickets[k]]
            assert got[t].position == c.position
            assert np.array_equal(alone.data(got[t]), d)


def test_device_queue_needs_a_gpu():
    from paper_1206_1187_amd import NNError
    with pytest.raises(NNError):
        serve.Server(np.array([orc.seed(wl.INDEX_MIN)], dtype=np.uint64), 1 << 20, fake=True,
                     device_queue=True)
