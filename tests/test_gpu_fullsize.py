"""Full-size GPU parity of exactly the launches the benchmark times.

The plain bulk workload (2^30 f64 variates, then 2^28 raw u64 states from
one seed index) in the launch configuration bench.py uses for each kind,
the batched workload (10,000 streams, 2.7e9 outputs) in the batch shape
bench.py uses, and the 3^40 generator's default launch for 2^30 f64
outputs (the bench's modulus-3^40 figure), each compared element by element
with the oracle.  The
configurations come from one place (``tune.BENCH_PLAIN`` and
``tune.bench_batch_kw``), which bench.py reads too.  Bit-exact: the path is
integer work and the variate is one IEEE multiplication (Section 2's
parallel sequence must equal the serial one).
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402
from paper_1206_1187_amd import tune  # noqa: E402

CHUNK = 1 << 25  # elements compared per host round trip


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    nn.init(0)
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _compare_chunks(flat, z0, count, kind, label):
    """flat: the int64 view of a cuda tensor holding z_1..z_count after z0;
    compared with the oracle CHUNK elements at a time (the oracle's chunk
    started by its own skip-ahead)."""
    host = np.empty(CHUNK, dtype=np.float64 if kind == "f64" else np.uint64)
    for c0 in range(0, count, CHUNK):
        n = min(CHUNK, count - c0)
        ref = host[:n]
        orc.gen_into(orc.skip(z0, c0), ref, threads=0)
        got = flat[c0:c0 + n].cpu().numpy().view(np.uint64)
        bad = np.nonzero(got != ref.view(np.uint64))[0]
        assert bad.size == 0, (label, c0, bad[:4], got[bad[:4]], ref.view(np.uint64)[bad[:4]])


@pytest.mark.parametrize("kind", ["f64", "u64"])
def test_bench_plain_launch_full_size_bit_exact(kind):
    """The benchmark's plain-bulk launch for `kind` at full size (the same
    seed index, count and nn_launch_cfg bench.py times), every output
    against the oracle."""
    case = wl.plain_bulk()
    count = case.count_f64 if kind == "f64" else case.count_u64
    cfg = tune.bench_plain_cfg(kind)
    _say("bench plain launch", kind, count, cfg.as_dict())
    z0 = nn.seed(case.index)
    assert z0 == orc.seed(case.index)
    dt = torch.float64 if kind == "f64" else torch.uint64
    out = torch.empty(count, dtype=dt, device="cuda")
    out.view(torch.int64).fill_(-1)
    zn = nn.generate_into(z0, out, cfg=cfg)
    torch.cuda.synchronize()
    assert zn == orc.skip(z0, count)
    _compare_chunks(out.view(torch.int64), z0, count, kind, "plain " + kind)
    del out
    torch.cuda.empty_cache()


def test_bench_batched_launch_full_size_bit_exact():
    """The batched workload in full: all 10,000 streams, every output, in
    the batch shape the benchmark replays, against the oracle stream by
    stream; plus the final states."""
    states, lengths, offsets = tune.batch_workload()
    total = int(lengths.sum())
    kw = tune.bench_batch_kw(total)
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    out.view(torch.int64).fill_(-1)
    with nn.BatchPlan("f64", len(states), total, **kw) as plan:
        _say("bench batched launch", plan.cfg().as_dict(), total)
        fin = plan.generate(states, lengths, offsets, out, final_states=True)
        torch.cuda.synchronize()
    flat = out.view(torch.int64)
    for i, (s, n) in enumerate(zip(states.tolist(), lengths.tolist())):
        assert int(fin[i]) == orc.skip(s, n), i
    # Streams are packed back to back: compare CHUNK-sized runs of whole
    # streams, each stream's oracle values written into its slot.
    host = np.empty(CHUNK + (1 << 22), dtype=np.float64)
    i, n_streams = 0, len(states)
    while i < n_streams:
        j, o0 = i, int(offsets[i])
        while j < n_streams and int(offsets[j]) + int(lengths[j]) - o0 <= host.size:
            j += 1
        end = int(offsets[j - 1]) + int(lengths[j - 1])
        for k in range(i, j):
            o, n = int(offsets[k]) - o0, int(lengths[k])
            orc.gen_into(int(states[k]), host[o:o + n], threads=0 if n > 1 << 16 else 1)
        got = flat[o0:end].cpu().numpy().view(np.uint64)
        ref = host[:end - o0].view(np.uint64)
        bad = np.nonzero(got != ref)[0]
        if bad.size:
            k = int(np.searchsorted(offsets, o0 + bad[0], side="right")) - 1
            raise AssertionError(("stream", k, "element", o0 + int(bad[0]) - int(offsets[k]),
                                  got[bad[0]], ref[bad[0]]))
        i = j
    del out, flat
    torch.cuda.empty_cache()


def test_e40_default_launch_full_size_bit_exact():
    """The 3^40 generator's default launch for 2^30 f64 outputs (the flat
    layout, 16 rows per chunk in XCD runs, FP64 limb step), every output against the
    3^40 oracle: slices of 2^26 filled on host threads, each from the
    oracle's own skip-ahead."""
    n = 1 << 30
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 123456789)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    out.view(torch.int64).fill_(-1)
    _say("e40 default launch, 2^30 f64")
    zn = nn.e40_generate_into(z0, out)
    torch.cuda.synchronize()
    assert zn == orc.e40_skip(z0, n)
    flat = out.view(torch.int64)
    piece = 1 << 26

    def ref(i):
        return orc.e40_gen(orc.e40_skip(z0, i * piece), piece, "f64")[0].view(np.uint64)

    with ThreadPoolExecutor(max_workers=min(16, orc.max_threads())) as ex:
        for i, want in enumerate(ex.map(ref, range(n // piece))):
            got = flat[i * piece:(i + 1) * piece].cpu().numpy().view(np.uint64)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, ("e40", i * piece + int(bad[0]), got[bad[0]], want[bad[0]])
    del out, flat
    torch.cuda.empty_cache()
