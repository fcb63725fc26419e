"""GPU tests of nn_generate_batch_static, the batched entry point that
allocates nothing (its workspace is the library's static device array):
two calls in a row, the second smaller, each compared bit for bit with
nn_generate_batch on a chunked plan (the entry point it is a variant of)
and with the oracle, including the gaps between windows."""
import sys

import numpy as np
import pytest

import oracle as orc
from paper_1206_1187_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402
from paper_1206_1187_amd import _native  # noqa: E402

SENTINEL = 0xDEADBEEFCAFEF00D


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bits(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def _sentinel(n):
    host = np.full(n, SENTINEL, dtype=np.uint64)
    return torch.from_numpy(host.view(np.int64)).cuda()


def _batch(seed, n, max_log2):
    """n streams with seeded states, lengths log-uniform in [1, 2^max_log2]
    (one of them empty), windows packed with gaps of 0..2 outputs from an odd
    offset, so window starts take every residue modulo the 2048-output
    chunks."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(wl.INDEX_MIN, wl.INDEX_MAX, n, endpoint=True, dtype=np.int64)
    states = np.array([orc.seed(int(a)) for a in idx], dtype=np.uint64)
    lengths = np.floor(np.exp(rng.uniform(0.0, max_log2 * np.log(2.0), n))).astype(np.uint64)
    lengths[n // 2] = 0
    gaps = rng.integers(0, 3, n)
    offsets = np.zeros(n, dtype=np.uint64)
    pos = 1
    for i in range(n):
        pos += int(gaps[i])
        offsets[i] = pos
        pos += int(lengths[i])
    return states, lengths, offsets, pos + 5


def _check_oracle(got, states, lengths, offsets, kind):
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


@pytest.mark.parametrize("kind", ["f64", "u64"])
def test_static_batch_matches_plan_two_calls(kind):
    """Call 1: 700 streams up to 2^18 outputs; call 2, right after on the
    same workspace: 40 streams up to 2^14.  Each against a chunked plan's
    nn_generate_batch and the oracle."""
    dt = torch.float64 if kind == "f64" else torch.uint64
    for call, (seed, n, lg) in enumerate([(71, 700, 18), (72, 40, 14)]):
        states, lengths, offsets, total = _batch(seed, n, lg)
        _say("static batch call %d: kind %s, %d streams, %d outputs" % (call, kind, n, total))
        got = _sentinel(total).view(dt)
        fin = nn.generate_batch_static(states, lengths, offsets, got, final_states=True)
        torch.cuda.synchronize()
        want = _sentinel(total).view(dt)
        with nn.BatchPlan(kind, n, int(lengths.sum()), chunks=True) as plan:
            fin_plan = plan.generate(states, lengths, offsets, want, final_states=True)
        torch.cuda.synchronize()
        g, w = _bits(got), _bits(want)
        bad = np.nonzero(g != w)[0]
        assert bad.size == 0, (call, bad[:8])
        assert np.array_equal(fin, fin_plan)
        assert fin.tolist() == [orc.skip(int(s), int(k)) for s, k in zip(states, lengths)]
        _check_oracle(g, states, lengths, offsets, kind)


def test_static_batch_empty_and_limits():
    """No streams, only empty windows: nothing written, states unchanged;
    more streams than the workspace holds: NN_ERANGE before any launch."""
    out = _sentinel(64).view(torch.float64)
    assert nn.generate_batch_static([], [], [], out, final_states=True).size == 0
    s = orc.seed(wl.INDEX_MIN)
    fin = nn.generate_batch_static([s, s], [0, 0], [3, 9], out, final_states=True)
    torch.cuda.synchronize()
    assert fin.tolist() == [s, s]
    assert (_bits(out) == SENTINEL).all()
    n = (1 << 16) + 1
    with pytest.raises(nn.NNError) as ei:
        nn.generate_batch_static([s] * n, [1] * n, list(range(n)),
                                 torch.empty(n, dtype=torch.float64, device="cuda"))
    assert ei.value.status == _native.NN_ERANGE
