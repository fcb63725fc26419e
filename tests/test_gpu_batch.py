"""GPU parity of the batched form (nn_generate_batch) against the oracle,
and against the plain path stream by stream.  Bit-exact throughout."""
import ctypes
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402

M = 3 ** 33
P = 2 * 3 ** 32
SENTINEL = 0xDEADBEEFCAFEF00D


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bits(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def _sentinel(n):
    host = np.full(n, SENTINEL, dtype=np.uint64)
    return torch.from_numpy(host.view(np.int64)).cuda()


def _mixed_batch(seed, lengths):
    """Random states, the given lengths, windows packed back to back with a
    gap of 0..2 elements (so offsets take both parities)."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(wl.INDEX_MIN, wl.INDEX_MAX, len(lengths), endpoint=True, dtype=np.int64)
    states = np.array([orc.seed(int(a)) for a in idx], dtype=np.uint64)
    lengths = np.asarray(lengths, dtype=np.uint64)
    gaps = rng.integers(0, 3, len(lengths)).astype(np.uint64)
    offsets = np.zeros(len(lengths), dtype=np.uint64)
    pos = 1  # the first window starts at an odd offset
    for i in range(len(lengths)):
        pos += int(gaps[i])
        offsets[i] = pos
        pos += int(lengths[i])
    return states, lengths, offsets, pos + 3


def _check_batch(got, states, lengths, offsets, kind):
    written = np.zeros(got.size, dtype=bool)
    for s, n, o in zip(states.tolist(), lengths.tolist(), offsets.tolist()):
        ref, _ = orc.gen(s, n, kind)
        assert np.array_equal(got[o:o + n], ref.view(np.uint64)), (s, n, o)
        written[o:o + n] = True
    assert (got[~written] == SENTINEL).all(), "write outside every window"


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    nn.init(0)
    yield
    torch.cuda.synchronize()


LENGTHS = [0, 1, 2, 3, 4, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 8191, 8192, 8193,
           16383, 16384, 16385, 70_001, 100_003, 262_145]


@pytest.mark.parametrize("kind", ["u64", "f64"])
@pytest.mark.parametrize("mulmod,interleaved", [("fp64", False), ("fp64", True), ("shoup", False),
                                                ("barrett", False), ("montgomery", False)])
def test_batch_bit_exact_mixed_lengths(kind, mulmod, interleaved):
    """Both batch kernels, every reduction, many shapes and cluster sizes."""
    states, lengths, offsets, total = _mixed_batch(11, LENGTHS)
    dt = torch.float64 if kind == "f64" else torch.uint64
    for block, grid, cluster, graph in [(256, 0, 0, True), (64, 3, 1, False), (1024, 7, 1, True),
                                        (128, 1, 1, True), (64, 1000, 8, True),
                                        (256, 4096, 4, True), (128, 12, 3, True),
                                        (256, 64, 64, False), (512, 5, 1, True)]:
        if interleaved and block not in (64, 128, 256):
            continue
        _say("batch", kind, mulmod, interleaved, block, grid, cluster, graph)
        buf = _sentinel(total)
        with nn.BatchPlan(kind, 64, total, block=block, grid=grid, cluster=cluster,
                          mulmod=mulmod, graph=graph, interleaved=interleaved) as plan:
            assert bool(plan.cfg().flags & 16) == interleaved
            fin = plan.generate(states, lengths, offsets, buf.view(dt), final_states=True)
            torch.cuda.synchronize()
        _check_batch(_bits(buf), states, lengths, offsets, kind)
        for s, n, f in zip(states.tolist(), lengths.tolist(), fin.tolist()):
            assert f == orc.skip(s, n)


@pytest.mark.parametrize("kind", ["u64", "f64"])
def test_chunked_batch_bit_exact_mixed_lengths(kind):
    """The chunked kernel (sorted windows: a record per 2048-output chunk,
    one workgroup writing every window's part of it; dealt round-robin to
    persistent workgroups when the grid is fixed): windows shorter than a chunk,
    several windows in one chunk, windows starting and ending inside chunks
    at both offset parities, gaps between windows; grids from one workgroup
    (every record on it) to more workgroups than records; graph and direct
    launches; temporal and non-temporal stores; residency caps from 2 to 16
    workgroups per compute unit."""
    lengths = LENGTHS + [2047, 2048, 2049, 4095, 4096, 4097, 6143, 1, 2, 5, 3000, 1, 1]
    states, lengths, offsets, total = _mixed_batch(13, lengths)
    dt = torch.float64 if kind == "f64" else torch.uint64
    for grid, graph, temporal, occ in [(0, True, False, 0), (1, True, False, 0),
                                       (3, False, True, 0), (7, True, True, 2),
                                       (1000, True, False, 0), (4096, False, False, 0),
                                       (0, True, True, 6), (0, False, False, 16)]:
        _say("chunked", kind, grid, graph, temporal, occ)
        buf = _sentinel(total)
        with nn.BatchPlan(kind, 64, total, grid=grid, graph=graph, temporal=temporal,
                          chunks=True, occupancy=occ) as plan:
            assert plan.cfg().flags & 32
            assert plan.cfg().occupancy == (occ or 4)
            fin = plan.generate(states, lengths, offsets, buf.view(dt), final_states=True)
            torch.cuda.synchronize()
        _check_batch(_bits(buf), states, lengths, offsets, kind)
        for s, n, f in zip(states.tolist(), lengths.tolist(), fin.tolist()):
            assert f == orc.skip(s, n)


@pytest.mark.parametrize("kind", ["u64", "f64"])
def test_chunked_batch_xcd_runs(kind):
    """Batches of more records than one XCD run (2048 chunk records): the
    chunk kernel takes whole runs XCD by XCD and the records after the last
    run in workgroup order.  Long windows over several runs mixed with short
    ones and windows sharing chunks; one workgroup per record and persistent
    grids that wrap around the records; against the oracle."""
    rng = np.random.default_rng(23)
    lengths = [3 * 2048 * 2048 + 5, 1, 2047, 777_777, 2048 * 2048 - 3] + \
        [int(x) for x in rng.integers(1, 5000, 40)] + [1_500_001, 9]
    states, lengths, offsets, total = _mixed_batch(29, lengths)
    dt = torch.float64 if kind == "f64" else torch.uint64
    for grid, temporal in [(0, True), (0, False), (1000, True), (4099, True)]:
        _say("chunked xcd runs", kind, grid, temporal, total)
        buf = _sentinel(total)
        with nn.BatchPlan(kind, 64, total, grid=grid, temporal=temporal, chunks=True) as plan:
            plan.generate(states, lengths, offsets, buf.view(dt))
            torch.cuda.synchronize()
        _check_batch(_bits(buf), states, lengths, offsets, kind)
        del buf


@pytest.mark.parametrize("graph", [True, False])
def test_chunked_batches_back_to_back(graph):
    """A chunked plan uploads each batch and runs its record pre-pass on a
    side stream, overlapping the previous batch's chunk kernel: six batches
    with different windows (both slots reused twice over, small batches that
    travel in the kernel arguments between them) enqueued back to back on
    one stream into separate outputs, with no host synchronization between
    them; every output against the oracle."""
    specs = [(31, [2048 * 2048 * 2 + 17, 5, 70_001, 4097]), (32, [3, 1, 2]),
             (33, [1_000_003, 2048 * 1500, 1, 64]), (34, [2047, 2049] * 20),
             (35, [12345]), (36, [2048 * 2048 * 3 + 1])]
    batches = [_mixed_batch(seed, lengths) for seed, lengths in specs]
    cap = max(b[3] for b in batches)
    bufs = [_sentinel(b[3]) for b in batches]
    with nn.BatchPlan("f64", 64, cap, graph=graph, chunks=True) as plan:
        for (states, lengths, offsets, total), buf in zip(batches, bufs):
            plan.generate(states, lengths, offsets, buf.view(torch.float64))
        torch.cuda.synchronize()
    for (states, lengths, offsets, total), buf in zip(batches, bufs):
        _check_batch(_bits(buf), states, lengths, offsets, "f64")


def test_chunked_batch_dense_short_windows():
    """Thousands of windows of 1 to 40 outputs packed back to back, so most
    chunks hold dozens of windows (all written by the chunk's one workgroup
    from the windows' first-chunk records), against the oracle."""
    rng = np.random.default_rng(17)
    lengths = [int(x) for x in rng.integers(1, 41, 3000)]
    states, lengths, offsets, total = _mixed_batch(18, lengths)
    buf = _sentinel(total)
    with nn.BatchPlan("f64", 4096, total, chunks=True) as plan:
        plan.generate(states, lengths, offsets, buf.view(torch.float64))
        torch.cuda.synchronize()
    _check_batch(_bits(buf), states, lengths, offsets, "f64")


@pytest.mark.parametrize("temporal", [False, True])
def test_chunked_batch_unsorted_windows(temporal):
    """Windows given out of output order (the same windows as the mixed
    batch, shuffled; the plan sorts them by output offset): against the
    oracle, final states in the caller's order, nothing written outside."""
    lengths = LENGTHS + [2047, 2048, 2049, 4097, 1, 2, 5, 3000, 1, 1]
    states, lengths, offsets, total = _mixed_batch(19, lengths)
    perm = np.random.default_rng(20).permutation(len(lengths))
    states, lengths, offsets = states[perm], lengths[perm], offsets[perm]
    buf = _sentinel(total)
    with nn.BatchPlan("f64", 64, total, chunks=True, temporal=temporal) as plan:
        fin = plan.generate(states, lengths, offsets, buf.view(torch.float64), final_states=True)
        torch.cuda.synchronize()
    _check_batch(_bits(buf), states, lengths, offsets, "f64")
    for s, n, f in zip(states.tolist(), lengths.tolist(), fin.tolist()):
        assert f == orc.skip(s, n)


def test_chunked_batch_validation():
    for bad in (dict(block=128), dict(cluster=4), dict(mulmod="shoup"), dict(interleaved=True)):
        with pytest.raises(nn.NNError):
            nn.BatchPlan("f64", 2, 1 << 20, chunks=True, **bad)


def test_graph_replays_with_eager_work_between():
    """Replay one plan's graph many times with other work and syncs in
    between; every replay must equal the oracle."""
    kind = "f64"
    with nn.BatchPlan(kind, 64, 1 << 22, grid=37) as plan:
        for rep in range(6):
            states, lengths, offsets, total = _mixed_batch(100 + rep, LENGTHS[rep:])
            buf = _sentinel(total)
            plan.generate(states, lengths, offsets, buf.view(torch.float64))
            # eager work on the same stream between replays
            junk = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
            nn.generate_into(orc.seed(wl.INDEX_MIN + rep), junk)
            junk.mul_(2.0)
            torch.cuda.synchronize()
            _check_batch(_bits(buf), states, lengths, offsets, kind)


def test_back_to_back_batches_without_sync():
    """Several batches of one plan enqueued before any host synchronisation."""
    bufs, cases = [], []
    with nn.BatchPlan("u64", 64, 1 << 21, block=512) as plan:
        for rep in range(5):
            states, lengths, offsets, total = _mixed_batch(200 + rep, LENGTHS)
            buf = _sentinel(total)
            plan.generate(states, lengths, offsets, buf.view(torch.uint64))
            bufs.append(buf)
            cases.append((states, lengths, offsets))
        torch.cuda.synchronize()
    for buf, (states, lengths, offsets) in zip(bufs, cases):
        _check_batch(_bits(buf), states, lengths, offsets, "u64")


def test_batch_equals_plain_per_stream():
    states, lengths, offsets, total = _mixed_batch(7, LENGTHS)
    buf = _sentinel(total)
    with nn.BatchPlan("f64", 64, total) as plan:
        plan.generate(states, lengths, offsets, buf.view(torch.float64))
    torch.cuda.synchronize()
    got = _bits(buf)
    for s, n, o in zip(states.tolist(), lengths.tolist(), offsets.tolist()):
        if n == 0:
            continue
        t, _ = nn.generate(s, n, "f64")
        torch.cuda.synchronize()
        assert np.array_equal(_bits(t), got[o:o + n])


def test_long_stream_split_boundary():
    """A stream longer than one internal piece (2^24 outputs)."""
    s = orc.seed(wl.INDEX_MIN + 4242)
    n = (1 << 24) * 2 + 777
    buf = _sentinel(n + 3)
    with nn.BatchPlan("u64", 4, n) as plan:
        fin = plan.generate([s], [n], [1], buf.view(torch.uint64), final_states=True)
    torch.cuda.synchronize()
    got = _bits(buf)
    assert got[0] == SENTINEL and (got[n + 1:] == SENTINEL).all()
    assert int(fin[0]) == orc.skip(s, n)
    for start in (0, (1 << 24) - 4096, (2 << 24) - 4096, n - 5000):
        k = min(8192, n - start)
        ref, _ = orc.gen(orc.skip(s, start), k, "u64")
        assert np.array_equal(got[1 + start:1 + start + k], ref), start


def test_batch_errors_enqueue_nothing():
    with nn.BatchPlan("f64", 2, 10_000) as plan:
        out = _sentinel(20_000)
        good = orc.seed(wl.INDEX_MIN)
        with pytest.raises(nn.NNError):  # too many streams
            plan.generate([good] * 3, [10] * 3, [0, 10, 20], out.view(torch.float64))
        with pytest.raises(nn.NNError):  # too many outputs
            plan.generate([good], [19_999], [0], out.view(torch.float64))
        with pytest.raises(nn.NNError):  # invalid state
            plan.generate([3], [10], [0], out.view(torch.float64))
        with pytest.raises(nn.NNError):  # misaligned output base
            plan.generate([good], [10], [0], out[1:].view(torch.float64))
        torch.cuda.synchronize()
        assert (_bits(out) == SENTINEL).all()
        fin = plan.generate([good], [0], [0], out.view(torch.float64), final_states=True)
        assert int(fin[0]) == good


def test_skip_stress_full_as_one_batch():
    """Config 3 in full: 65,536 offsets over the whole period (forced ones
    next to the wrap), 4,096 variates each, one batched launch."""
    base = orc.seed(wl.INDEX_MIN)
    offs = wl.skip_offsets()
    states = np.array([nn.skip(base, int(o)) for o in offs], dtype=np.uint64)
    lengths = np.full(offs.size, 4096, dtype=np.uint64)
    offsets = np.arange(offs.size, dtype=np.uint64) * 4096
    out = torch.empty(offs.size * 4096, dtype=torch.float64, device="cuda")
    with nn.BatchPlan("f64", offs.size, out.numel()) as plan:
        plan.generate(states, lengths, offsets, out)
    torch.cuda.synchronize()
    got = _bits(out).reshape(offs.size, 4096)
    for i, o in enumerate(offs.tolist()):
        z = orc.skip(base, o)
        assert int(states[i]) == z
        ref, _ = orc.gen(z, 4096, "f64")
        assert np.array_equal(got[i], ref.view(np.uint64)), (i, o)


@pytest.mark.parametrize("shape", ["blocked", "interleaved", "tuned", "tuned-", "tuned+"])
def test_batched_workload_full_size_sampled(shape):
    """Config 4 at full size (10,000 streams, 2.7e9 outputs): both batch
    kernels at their default shapes, and the tuned shape the benchmark runs
    with the neighbouring grids it may pick instead (cluster kept): every
    stream's first and last 64 outputs, and 400 whole streams, against the
    oracle."""
    from paper_1206_1187_amd import tune
    case = wl.batched()
    states = np.array([orc.seed(int(a)) for a in case.indices], dtype=np.uint64)
    lengths = case.lengths
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    total = int(lengths.sum())
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    if shape in ("blocked", "interleaved"):
        kw = dict(interleaved=shape == "interleaved")
    else:
        kw = tune.best_batch_cfg("f64", total)
        if shape != "tuned" and kw.get("grid"):
            step = max(16, int(kw.get("cluster") or 16))
            kw = dict(kw, grid=kw["grid"] + (step if shape == "tuned+" else -step))
    with nn.BatchPlan("f64", len(states), total, **kw) as plan:
        _say("batched full", shape, plan.cfg().as_dict(), total)
        fin = plan.generate(states, lengths, offsets, out, final_states=True)
    torch.cuda.synchronize()
    flat = out.view(torch.int64)
    rng = np.random.default_rng(99)
    whole = set(rng.choice(len(states), 400, replace=False).tolist())
    for i, (s, n, o) in enumerate(zip(states.tolist(), lengths.tolist(), offsets.tolist())):
        assert int(fin[i]) == orc.skip(s, n)
        if i in whole:
            ref, _ = orc.gen(s, n, "f64", threads=0 if n > 1 << 16 else 1)
            got = flat[o:o + n].cpu().numpy().view(np.uint64)
            assert np.array_equal(got, ref.view(np.uint64)), i
        else:
            k = min(64, n)
            head, _ = orc.gen(s, k, "f64")
            tail, _ = orc.gen(orc.skip(s, n - k), k, "f64")
            assert np.array_equal(flat[o:o + k].cpu().numpy().view(np.uint64),
                                  head.view(np.uint64)), i
            assert np.array_equal(flat[o + n - k:o + n].cpu().numpy().view(np.uint64),
                                  tail.view(np.uint64)), i
    del out, flat
    torch.cuda.empty_cache()


def test_slots_alternate_across_streams():
    """Back-to-back batches of one plan on three different streams: the plan
    alternates two staging slots, and a slot is reused only after the batch
    that last used it has finished, whatever stream it ran on."""
    streams = [torch.cuda.Stream() for _ in range(3)]
    bufs, cases = [], []
    with nn.BatchPlan("f64", 64, 1 << 21) as plan:
        for rep in range(7):
            states, lengths, offsets, total = _mixed_batch(300 + rep, LENGTHS)
            buf = _sentinel(total)
            torch.cuda.synchronize()
            s = streams[rep % 3]
            plan.generate(states, lengths, offsets, buf.view(torch.float64), stream=s)
            bufs.append(buf)
            cases.append((states, lengths, offsets))
        torch.cuda.synchronize()
    for buf, (states, lengths, offsets) in zip(bufs, cases):
        _check_batch(_bits(buf), states, lengths, offsets, "f64")


@pytest.mark.parametrize("kind", ["u64", "f64"])
@pytest.mark.parametrize("mulmod,interleaved", [("fp64", False), ("shoup", False),
                                                ("barrett", False), ("montgomery", False),
                                                ("fp64", True)])
def test_small_batches_in_kernel_arguments(kind, mulmod, interleaved):
    """Batches of up to 16 windows travel in the kernel arguments (no
    upload) and run the blocked kernel, also in an interleaved plan (whose
    workgroups then form one cluster); 1, 2, 15, 16 and 17 windows (17 takes
    the workspace path), odd offsets, ragged lengths, one window long enough
    to be split in pieces."""
    dt = torch.float64 if kind == "f64" else torch.uint64
    lengths_all = [1, 511, 512, 513, 70_001, 3, 1024, 8193, 2, 65, 100_003, 17, 4096, 9, 300, 1025,
                   33]
    with nn.BatchPlan(kind, 32, 1 << 26, mulmod=mulmod, block=128, grid=9,
                      interleaved=interleaved) as plan:
        for nwin in (1, 2, 15, 16, 17):
            states, lengths, offsets, total = _mixed_batch(400 + nwin, lengths_all[:nwin])
            _say("inline", kind, mulmod, "interleaved" if interleaved else "blocked", nwin)
            buf = _sentinel(total)
            fin = plan.generate(states, lengths, offsets, buf.view(dt), final_states=True)
            torch.cuda.synchronize()
            _check_batch(_bits(buf), states, lengths, offsets, kind)
            for s, n, f in zip(states.tolist(), lengths.tolist(), fin.tolist()):
                assert f == orc.skip(s, n)
        # one stream of 2^25 + 5 outputs: three pieces, still inline
        s0 = orc.seed(wl.INDEX_MIN + 77)
        n = (1 << 25) + 5
        buf = _sentinel(n + 2)
        plan.generate([s0], [n], [1], buf.view(dt))
        torch.cuda.synchronize()
        got = _bits(buf)
        assert got[0] == SENTINEL and got[n + 1] == SENTINEL
        for start in (0, (1 << 24) - 3, (1 << 25) - 8):
            ref, _ = orc.gen(orc.skip(s0, start), 13, kind)
            assert np.array_equal(got[1 + start:1 + start + 13], ref.view(np.uint64)), start


def test_batch_offsets_beyond_32_bit_indexing():
    """Windows whose output offsets lie past 2^32 elements (a 34 GiB output),
    one of them at an odd offset, in the workspace and the kernel-argument
    paths."""
    base = (1 << 32) + 1
    lengths = [5000, 1 << 20, 77, 300_001]
    offsets = [base, base + 5000 + 3, base + 5000 + 3 + (1 << 20) + 1, 3]
    total = offsets[2] + lengths[2] + 16
    states = [orc.seed(wl.INDEX_MIN + 31 * i) for i in range(4)]
    out = torch.empty(total, dtype=torch.uint64, device="cuda")
    for graph, il in ((True, False), (False, False), (True, True)):
        _say("beyond 2^32", "graph" if graph else "direct", "interleaved" if il else "blocked")
        with nn.BatchPlan("u64", 32, total, graph=graph, interleaved=il) as plan:
            plan.generate(states, lengths, offsets, out)
            torch.cuda.synchronize()
        flat = out.view(torch.int64)
        for s, n, o in zip(states, lengths, offsets):
            for st in (0, n - 64):
                ref, _ = orc.gen(orc.skip(s, st), 64, "u64")
                got = flat[o + st:o + st + 64].cpu().numpy().view(np.uint64)
                assert np.array_equal(got, ref), (o, st)
        # more than 16 windows: the workspace path with the same offsets
        st2 = states * 5
        ln2 = [64] * 20
        of2 = [base + 128 * i + (i & 1) for i in range(20)]
        with nn.BatchPlan("u64", 32, total, graph=graph, interleaved=il) as plan:
            plan.generate(st2, ln2, of2, out)
            torch.cuda.synchronize()
        for s, o in zip(st2, of2):
            ref, _ = orc.gen(s, 64, "u64")
            got = out.view(torch.int64)[o:o + 64].cpu().numpy().view(np.uint64)
            assert np.array_equal(got, ref), o
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("grid,temporal", [(1, False), (3, False), (3, True)])
def test_interleaved_record_chunks(grid, temporal):
    """The interleaved kernel stages row records in LDS 4096 at a time (the
    first chunk shorter on most workgroups): workgroups with well over 4096
    rows, windows at both offset parities, against the oracle; non-temporal
    and temporal stores."""
    rng = np.random.default_rng(40 + grid)
    lengths = [int(x) for x in rng.integers(1, 100_000, 90)] + [300_001]
    states, lengths, offsets, total = _mixed_batch(41 + grid, lengths)
    buf = _sentinel(total)
    with nn.BatchPlan("f64", 128, total, block=64, grid=grid, interleaved=True,
                      temporal=temporal) as plan:
        rows = sum((int(n) + (int(o) % 128) + 127) // 128 for n, o in zip(lengths, offsets))
        _say("interleaved chunks", grid, "temporal" if temporal else "nt", "rows", rows)
        assert rows // grid > 2 * 4096
        plan.generate(states, lengths, offsets, buf.view(torch.float64))
        torch.cuda.synchronize()
    _check_batch(_bits(buf), states, lengths, offsets, "f64")


def test_interleaved_output_index_limit():
    """The interleaved kernel's shapes (FP64, block 64, 128 or 256, clusters dividing the grid),
    and its row records' 52-bit output indices: windows reaching past 2^51
    elements are refused before anything is enqueued."""
    good = orc.seed(wl.INDEX_MIN)
    out = _sentinel(64)
    from paper_1206_1187_amd import _native
    for bad in (dict(block=192), dict(block=512), dict(mulmod="shoup"), dict(grid=128, cluster=3)):
        with pytest.raises(nn.NNError):
            nn.BatchPlan("f64", 2, 1 << 20, interleaved=True, **bad)
    with nn.BatchPlan("f64", 32, 1 << 20, interleaved=True) as plan:
        # through the C ABI (the binding already refuses windows past its
        # tensor), with more windows than travel in the kernel arguments, so
        # the batch goes to the interleaved kernel, which refuses it before
        # anything is enqueued
        n = 18
        descs = (_native.StreamDesc * n)(*([(good, 2, 2 * i) for i in range(n - 1)] +
                                           [(good, 10, (1 << 51) - 5)]))
        rc = _native.lib().nn_generate_batch(plan._h, ctypes.cast(descs, ctypes.c_void_p), n,
                                             ctypes.c_void_p(out.data_ptr()), None, None)
        assert rc == _native.NN_ERANGE
        assert b"2^51" in _native.lib().nn_last_error()
        plan.generate([good], [64], [0], out.view(torch.float64))
        torch.cuda.synchronize()
    ref, _ = orc.gen(good, 64, "f64")
    assert np.array_equal(_bits(out), ref.view(np.uint64))
