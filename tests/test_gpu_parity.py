"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exactness for raw states and for the
binary64 variates.  Inputs come from the seeded workload recipes; expected
values only from the oracle.
"""
import itertools
import math
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
VARIANTS = ["fp64", "barrett", "shoup", "montgomery"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bits(t):
    """Host uint64 view of the bits of a uint64/float64 cuda tensor."""
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def _sentinel_buffer(n):
    host = np.full(n, SENTINEL, dtype=np.uint64)
    return torch.from_numpy(host.view(np.int64)).cuda()


def _gen_guarded(state, count, kind, cfg=None, guard=4096):
    """Generate into the middle of a sentinel-filled buffer; check the guards."""
    dt = torch.float64 if kind == "f64" else torch.uint64
    buf = _sentinel_buffer(count + 2 * guard)
    view = buf[guard:guard + count].view(dt)
    new_state = nn.generate_into(state, view, cfg=cfg)
    torch.cuda.synchronize()
    got = _bits(buf)
    assert (got[:guard] == SENTINEL).all(), "write before the output"
    assert (got[guard + count:] == SENTINEL).all(), "write past the output"
    return got[guard:guard + count], new_state


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    nn.init(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["u64", "f64"])
def test_plain_single_bit_exact(kind):
    """2^20 outputs from seed index 3^33+100: exact vs the oracle; the first
    outputs also against the alpha digit sum at positions a + 53k."""
    case = wl.plain_single()
    _say("plain_single", kind, case.index)
    z0 = nn.seed(case.index)
    assert z0 == orc.seed(case.index)
    got, zn = _gen_guarded(z0, case.count_u64, kind)
    ref, zr = orc.gen(z0, case.count_u64, kind, threads=0)
    assert zn == zr
    bad = np.nonzero(got != ref.view(np.uint64))[0]
    assert bad.size == 0, (bad[:8], got[bad[:8]], ref.view(np.uint64)[bad[:8]])
    for k in range(1, 65):
        want = orc.digit_sum(case.index + 53 * k)
        if kind == "u64":
            assert int(got[k - 1]) == want
        else:
            assert got[k - 1] == np.float64(orc.to_f64(want)).view(np.uint64)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("kind", ["u64", "f64"])
def test_every_reduction_bit_exact(variant, kind):
    z0 = orc.seed(wl.plain_bulk().index)
    count = 3 * 65536 + 4099  # several rows of a 64K-thread grid plus a ragged tail
    ref, zr = orc.gen(z0, count, kind, threads=0)
    for block, grid, unroll in [(256, 256, 4), (64, 7, 1), (1024, 3, 8), (128, 1001, 2)]:
        for width, ilp in ((1, 1), (2, 1), (2, 2), (2, 4)):
            cfg = nn.make_cfg(block=block, grid=grid, mulmod=variant, unroll=unroll, width=width,
                              ilp=ilp)
            _say("reduction", variant, kind, block, grid, unroll, width, ilp)
            got, zn = _gen_guarded(z0, count, kind, cfg=cfg)
            assert zn == zr
            assert np.array_equal(got, ref.view(np.uint64)), (variant, kind, block, grid,
                                                              unroll, width, ilp)


@pytest.mark.parametrize("block", [64, 128, 256, 512, 1024])
def test_thread_count_independence(block):
    """The same serial sequence for any launch shape, count and tail."""
    z0 = orc.seed(wl.INDEX_MIN + 12345)
    ref_all, _ = orc.gen(z0, 300_000, "f64", threads=0)
    ref_all = ref_all.view(np.uint64)
    for grid in (1, 3, 64, 257):
        T = grid * block
        for width, ilp in ((1, 1), (2, 1), (2, 2), (2, 4)):
            row = T * width
            counts = {1, 2, 3, row - 1, row, row + 1, 3 * row + 17, 5 * row - 1, 99991}
            for count in sorted(counts):
                if count < 1 or count > ref_all.size:
                    continue
                for unroll in (1, 8):
                    cfg = nn.make_cfg(block=block, grid=grid, unroll=unroll, width=width,
                                      ilp=ilp)
                    got, zn = _gen_guarded(z0, count, "f64", cfg=cfg, guard=256)
                    assert np.array_equal(got, ref_all[:count]), (block, grid, count, unroll,
                                                                  width, ilp)
                    assert zn == orc.skip(z0, count)


def test_output_alignment():
    """An output that is only 8-byte aligned takes the flat layout by
    default, its first element from a one-workgroup launch and the rest
    16-byte aligned (also explicitly, in both kinds, with ragged tails, past
    the XCD runs, and for the fill); the row layout takes 8-byte stores
    there, and asking it for 16-byte stores is an error that writes nothing."""
    z0 = orc.seed(wl.INDEX_MIN + 99)
    ref, zr = orc.gen(z0, 50_001, "u64", threads=0)
    got, zn = _gen_guarded(z0, 50_001, "u64", guard=4097)
    assert np.array_equal(got, ref) and zn == zr
    big = 2 * 2048 * 2048 + 3 * 2048 + 3
    ref_u, _ = orc.gen(z0, big, "u64", threads=0)
    ref_f, _ = orc.gen(z0, big, "f64", threads=0)
    for cfg in (None, nn.make_cfg(layout="flat"), nn.make_cfg(layout="flat", unroll=1),
                nn.make_cfg(layout="rows")):
        for count in (1, 2, 3, 2048, 2049, 4097, big):
            for kind, r in (("u64", ref_u), ("f64", ref_f)):
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=513)
                assert np.array_equal(got, r.view(np.uint64)[:count]), (cfg, count, kind)
                assert zn == orc.skip(z0, count)
    for count in (1, 2, 4097, big):
        buf = _sentinel_buffer(count + 2 * 513)
        nn.fill(buf[513:513 + count], 0x3FF0000000000001, cfg=nn.make_cfg(layout="flat"))
        torch.cuda.synchronize()
        h = _bits(buf)
        assert (h[:513] == SENTINEL).all() and (h[513 + count:] == SENTINEL).all()
        assert (h[513:513 + count] == 0x3FF0000000000001).all()
    buf = _sentinel_buffer(50_001 + 2)
    with pytest.raises(nn.NNError):
        nn.generate_into(z0, buf[1:50_002].view(torch.uint64), cfg=nn.make_cfg(width=2))
    torch.cuda.synchronize()
    assert (_bits(buf) == SENTINEL).all()


@pytest.mark.parametrize("variant", VARIANTS)
def test_flat_layout_bit_exact(variant):
    """The flat layout (workgroups of 1-16 rows of 512 outputs) for every
    reduction, both kinds, ragged tails around the row and chunk sizes,
    residency caps and both store policies."""
    z0 = orc.seed(wl.INDEX_MIN + 31337)
    ref_u, _ = orc.gen(z0, 300_000, "u64", threads=0)
    ref_f, _ = orc.gen(z0, 300_000, "f64", threads=0)
    counts = (1, 2, 3, 511, 512, 513, 1023, 1024, 1025, 3 * 512 + 1, 2047, 2048, 2049, 8191,
              8193, 99_991, 300_000)
    for rows in (0, 1, 2, 4, 16):
        for count in counts:
            for occ in (0, 3):
                cfg = nn.make_cfg(mulmod=variant, layout="flat", occupancy=occ, unroll=rows)
                for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                    _say("flat", variant, rows, count, occ, kind)
                    got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=512)
                    assert np.array_equal(got, ref.view(np.uint64)[:count]), \
                        (variant, rows, count, occ, kind)
                    assert zn == orc.skip(z0, count)
        # both store policies write the same values
        for temporal in (True, False):
            cfg = nn.make_cfg(mulmod=variant, layout="flat", unroll=rows, temporal=temporal)
            got, _ = _gen_guarded(z0, 99_991, "f64", cfg=cfg)
            assert np.array_equal(got, ref_f.view(np.uint64)[:99_991]), (rows, temporal)


def test_flat_residency_cap_bounds():
    """The flat layout at the residency caps' bounds, 2 and 16 workgroups
    per compute unit (the LDS that a workgroup reserves is largest at 2),
    four and eight rows, both kinds, a count with whole XCD runs, leftover
    chunks and a ragged tail, against the oracle element by element."""
    z0 = orc.seed(wl.INDEX_MIN + 4242)
    count = 2048 * 2048 + 5 * 2048 + 777
    ref_u, _ = orc.gen(z0, count, "u64", threads=0)
    ref_f, _ = orc.gen(z0, count, "f64", threads=0)
    for occ in (2, 16):
        for rows in (4, 8):
            cfg = nn.make_cfg(layout="flat", unroll=rows, occupancy=occ)
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                _say("flat cap", occ, rows, kind)
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=512)
                assert np.array_equal(got, ref.view(np.uint64)), (occ, rows, kind)
                assert zn == orc.skip(z0, count)


@pytest.mark.parametrize("variant", ["fp64", "shoup"])
def test_flat_xcd_runs_bit_exact(variant):
    """Four-row flat launches take their whole chunks in XCD runs of 2048
    chunks (4,194,304 outputs), then the chunks after the last run in
    workgroup order from their own start, then the ragged tail: counts below,
    at and past one run, runs plus leftover chunks plus a tail, both kinds,
    against the oracle element by element."""
    run = 2048 * 2048
    z0 = orc.seed(wl.INDEX_MIN + 271828)
    top = 3 * run + 2047 * 2048 + 2047
    ref_u, _ = orc.gen(z0, top, "u64", threads=0)
    ref_f, _ = orc.gen(z0, top, "f64", threads=0)
    counts = (run - 2048, run - 1, run, run + 1, run + 2048, 2 * run + 7 * 2048 + 1234, top)
    for count in counts:
        for kind, ref in (("u64", ref_u), ("f64", ref_f)):
            for order in (False, True):  # XCD runs, then NN_CFG_ADDRESS_ORDER
                cfg = nn.make_cfg(mulmod=variant, layout="flat", unroll=4, occupancy=4,
                                  temporal=True, address_order=order)
                _say("flat xcd runs", variant, count, kind, order)
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=512)
                assert np.array_equal(got, ref.view(np.uint64)[:count]), (variant, count, kind)
                assert zn == orc.skip(z0, count)


def test_pick_plain_layout_returns_a_working_cfg():
    """tune.pick_plain_layout times the row and flat layouts and returns the
    faster; whichever it returns writes the oracle's values."""
    from paper_1206_1187_amd import tune
    z0 = orc.seed(wl.INDEX_MIN + 777)
    n = 1 << 20
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    rows = nn.make_cfg(layout="rows")
    cfg, times = tune.pick_plain_layout(rows, out, z0, rounds=1, reps=2)
    assert set(times) == {"rows", "flat"} and all(t > 0 for t in times.values())
    zn = nn.generate_into(z0, out, cfg=cfg)
    torch.cuda.synchronize()
    assert zn == orc.skip(z0, n)
    ref, _ = orc.gen(z0, 8192, "f64", threads=0)
    assert np.array_equal(_bits(out)[:8192], ref.view(np.uint64))
    # an output that is only 8-byte aligned: both layouts are timed there too
    cfg2, times2 = tune.pick_plain_layout(rows, out[1:], z0, rounds=1, reps=2)
    assert set(times2) == {"rows", "flat"}
    zn = nn.generate_into(z0, out[1:], cfg=cfg2)
    torch.cuda.synchronize()
    assert zn == orc.skip(z0, n - 1)
    assert np.array_equal(_bits(out)[1:8193], ref.view(np.uint64))


def test_config_validation():
    z0 = orc.seed(wl.INDEX_MIN)
    out = torch.empty(4096, dtype=torch.float64, device="cuda")
    bad = [nn.make_cfg(layout="flat", block=512), nn.make_cfg(layout="flat", width=1),
           nn.make_cfg(block=100), nn.make_cfg(block=2048), nn.make_cfg(unroll=3),
           nn.make_cfg(width=3), nn.make_cfg(occupancy=1), nn.make_cfg(occupancy=17),
           nn.make_cfg(layout="rows", occupancy=4), nn.make_cfg(mulmod=9),
           nn.make_cfg(ilp=3), nn.make_cfg(width=1, ilp=2), nn.make_cfg(layout="flat", ilp=2),
           nn.make_cfg(grid=1 << 20, block=1024), nn.make_cfg(layout="flat", unroll=3),
           nn.make_cfg(layout="flat", unroll=32), nn.make_cfg(layout="flat", grid=4),
           nn.make_cfg(layout="rows", address_order=True),
           nn.make_cfg(layout="consecutive", address_order=True)]
    both = nn.make_cfg(layout="flat", temporal=True)
    both.flags |= nn._native.NN_CFG_NONTEMPORAL_STORES
    bad.append(both)
    for cfg in bad:
        with pytest.raises(nn.NNError):
            nn.generate_into(z0, out, cfg=cfg)
    with pytest.raises(nn.NNError):
        nn.fill(out, 0, cfg=nn.make_cfg(layout="flat", unroll=3))
    with pytest.raises(nn.NNError):  # the row layout's 16-byte stores need 16-byte alignment
        nn.generate_into(z0, out[1:].view(torch.float64), cfg=nn.make_cfg(layout="rows", width=2))
    # the default for an aligned output is the flat layout; a row-only field
    # (block, grid, ilp, width 1) selects the row layout
    d = nn.default_cfg("f64", 1 << 30)
    assert d.flags & nn._native.NN_CFG_FLAT and d.width == 2 and d.block == 256
    assert d.unroll == 4 and d.occupancy == 4 and d.flags & nn._native.NN_CFG_TEMPORAL_STORES


def test_chained_calls_concatenate():
    z = orc.seed(wl.plain_bulk().index)
    parts, state = [], z
    for n in (1, 4097, 65536, 3, 100_000):
        t, state = nn.generate(state, n, "u64")
        parts.append(t)
    torch.cuda.synchronize()
    got = np.concatenate([_bits(t) for t in parts])
    ref, zr = orc.gen(z, got.size, "u64", threads=0)
    assert np.array_equal(got, ref) and state == zr


@pytest.mark.parametrize("state", [1, 2, M - 1, M - 2, M // 2, 4])
def test_extreme_states(state):
    if state % 3 == 0:
        pytest.skip("not a unit")
    for kind in ("u64", "f64"):
        got, zn = _gen_guarded(state, 70_001, kind)
        ref, zr = orc.gen(state, 70_001, kind, threads=0)
        assert np.array_equal(got, ref.view(np.uint64)) and zn == zr


def test_deterministic_and_nontemporal_agnostic():
    z = orc.seed(wl.INDEX_MIN + 7)
    a, _ = _gen_guarded(z, 500_000, "f64")
    b, _ = _gen_guarded(z, 500_000, "f64", cfg=nn.make_cfg(temporal=True))
    c, _ = _gen_guarded(z, 500_000, "f64")
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_skip_stress_sample():
    """Offsets over the whole period (incl. next to the wrap): state by
    skip-ahead, then 4,096 consecutive variates each (plain path)."""
    base = orc.seed(wl.INDEX_MIN)
    offs = wl.skip_offsets()
    pick = np.concatenate([offs[:64], offs[-64:], offs[64:-64][::509]])
    _say("skip_stress sample of", pick.size)
    outs = []
    for o in pick.tolist():
        s = nn.skip(base, o)
        assert s == orc.skip(base, o)
        t, _ = nn.generate(s, 4096, "f64")
        outs.append(t)
    torch.cuda.synchronize()
    for o, t in zip(pick.tolist(), outs):
        ref, _ = orc.gen(orc.skip(base, o), 4096, "f64")
        assert np.array_equal(_bits(t), ref.view(np.uint64)), o


def test_fill_ceiling_kernel_pattern():
    cfgs = [nn.make_cfg(block=block, grid=grid, width=width)
            for block, grid, width in [(256, 2048, 1), (64, 5, 1), (256, 256, 2), (64, 5, 2)]]
    cfgs += [nn.make_cfg(layout="flat", unroll=rows, occupancy=occ, temporal=t)
             for rows, occ, t in [(0, 0, None), (1, 3, None), (4, 4, True), (16, 0, False)]]
    for cfg, count in itertools.product(cfgs, (1 << 20, 100_003, 2049, 3)):
        if cfg is cfgs[6] and count == 1 << 20:
            count = 2 * 2048 * 2048 + 3 * 2048 + 5  # XCD runs, leftover chunks, tail
        buf = _sentinel_buffer(count + 512)
        nn.fill(buf[256:256 + count], 0x3FF0000000000001, cfg=cfg)
        torch.cuda.synchronize()
        h = _bits(buf)
        assert (h[:256] == SENTINEL).all() and (h[256 + count:] == SENTINEL).all()
        assert (h[256:256 + count] == 0x3FF0000000000001).all()
    # the fill that keeps the generator's start (flat layout only), past one
    # launch's 2^30 outputs so the chunk tables' last entries are read
    for cfg, count in [(cfgs[6], (1 << 30) + 4099), (cfgs[5], 100_003), (cfgs[7], 2049)]:
        buf = _sentinel_buffer(count + 512)
        nn.fill(buf[256:256 + count], 0x3FF0000000000001, cfg=cfg, with_start=True)
        torch.cuda.synchronize()
        h = _bits(buf)
        assert (h[:256] == SENTINEL).all() and (h[256 + count:] == SENTINEL).all()
        assert (h[256:256 + count] == 0x3FF0000000000001).all()
        del buf, h
    with pytest.raises(nn.NNError):
        nn.fill(torch.empty(1024, dtype=torch.float64, device="cuda"), 0, cfg=cfgs[0],
                with_start=True)


def test_plain_bulk_full_size_bit_exact():
    """The plain bulk workload at full size (2^30 f64 then 2^28 u64 from one
    seed index) through nn_generate with no configuration (the library's
    default launch), compared in full with the oracle chunk by chunk.  The
    benchmark's own launch configurations are compared in
    test_gpu_fullsize.py."""
    case = wl.plain_bulk()
    z0 = nn.seed(case.index)
    chunk = 1 << 25
    for kind, count in (("f64", case.count_f64), ("u64", case.count_u64)):
        _say("plain_bulk", kind, count, nn.default_cfg(kind, count).as_dict())
        out, zn = nn.generate(z0, count, kind)
        torch.cuda.synchronize()
        assert zn == orc.skip(z0, count)
        flat = out.view(torch.int64)
        host = np.empty(chunk, dtype=np.float64 if kind == "f64" else np.uint64)
        for c in range(count // chunk):
            zc = orc.skip(z0, c * chunk)
            orc.gen_into(zc, host, threads=0)
            got = flat[c * chunk:(c + 1) * chunk].cpu().numpy().view(np.uint64)
            bad = np.nonzero(got != host.view(np.uint64))[0]
            assert bad.size == 0, (kind, c, bad[:4])
        del out, flat
        torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,deltas", [("f64", (0, -16, 16)), ("u64", (0, -32, 32))])
def test_plain_bulk_full_size_row_grids_sampled(kind, deltas):
    """The row layout at full size in its tuned shape and with the
    neighbouring grids tune.pick_plain_grid chooses among: sampled chunks (the
    start, the ragged end, and random offsets) against the oracle."""
    from paper_1206_1187_amd import tune
    case = wl.plain_bulk()
    z0 = nn.seed(case.index)
    count = case.count_f64 if kind == "f64" else case.count_u64
    kw = tune.best_plain_cfg(kind, count, layout="rows")
    base = nn.make_cfg(**dict(kw, layout="rows", grid=kw.get("grid") or 128))
    dt = torch.float64 if kind == "f64" else torch.uint64
    out = torch.empty(count, dtype=dt, device="cuda")
    rng = np.random.default_rng(5)
    n = 1 << 16
    starts = [0, count - n] + [int(x) for x in rng.integers(0, count - n, 14)]
    for d in deltas:
        cfg = nn.LaunchCfg(*[getattr(base, f) for f, _ in base._fields_])
        cfg.grid = base.grid + d
        _say("bench grid", kind, cfg.as_dict())
        out.fill_(0)
        zn = nn.generate_into(z0, out, cfg=cfg)
        torch.cuda.synchronize()
        assert zn == orc.skip(z0, count)
        flat = out.view(torch.int64)
        for st in starts:
            ref, _ = orc.gen(orc.skip(z0, st), n, kind)
            got = flat[st:st + n].cpu().numpy().view(np.uint64)
            assert np.array_equal(got, ref.view(np.uint64)), (kind, d, st)
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("layout,rows", [(None, 0), ("flat", 4), ("flat", 16)])
def test_flat_chunk_boundary_beyond_one_launch(layout, rows):
    """Counts above one flat launch (2^30 outputs) are split into several
    launches; check the outputs on both sides of every split and the tail
    (and the default layout at the same count)."""
    z0 = orc.seed(wl.plain_bulk().index + 5)
    count = (1 << 30) + 4099
    _say("beyond one launch", layout, rows)
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    zn = nn.generate_into(z0, out, cfg=nn.make_cfg(layout=layout, unroll=rows))
    torch.cuda.synchronize()
    assert zn == orc.skip(z0, count)
    flat = out.view(torch.int64)
    for start, n in ((0, 8192), ((1 << 30) - 8192, 8192 + 4099), (123_456_789, 4096)):
        ref, _ = orc.gen(orc.skip(z0, start), n, "f64", threads=0)
        got = flat[start:start + n].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref.view(np.uint64)), start
    del out, flat
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mulmod", VARIANTS)
def test_fused_consumer_state_sum_exact(mulmod):
    """nn_consume: the sum of the raw states modulo 2^64 is exact for any
    launch shape.  The variate sum is a floating sum in an order the launch
    decides (lane sums, a wave reduction, atomics), so it is checked against
    the correctly rounded sum of the oracle's variates (math.fsum) within the
    error bound of summing n positive terms in any order: (n - 1) * 2^-53 of
    the sum, plus the final rounding of the reference.  The variates
    themselves are the bit-exact ones of the plain path."""
    z0 = orc.seed(wl.plain_bulk().index + 17)
    for count, block, grid in [(1, 0, 0), (1023, 64, 3), (300_001, 256, 7), (1 << 22, 0, 0),
                               (5_000_000, 512, 129)]:
        ref, zr = orc.gen(z0, count, "u64", threads=0)
        want = int(ref.sum(dtype=np.uint64))  # numpy wraps modulo 2^64
        cfg = nn.make_cfg(block=block, grid=grid, mulmod=mulmod)
        res, zn = nn.consume(z0, count, "u64", cfg=cfg)
        torch.cuda.synchronize()
        assert int(res.view(torch.int64).cpu().numpy().view(np.uint64)[0]) == want
        assert zn == zr
        resf, _ = nn.consume(z0, count, "f64", cfg=cfg)
        torch.cuda.synchronize()
        reff, _ = orc.gen(z0, count, "f64", threads=0)
        exact = math.fsum(reff.tolist())
        bound = (count - 1) * 2.0 ** -53 * exact + 2.0 ** -52 * exact
        assert abs(float(resf.cpu()[0]) - exact) <= bound, (count, float(resf.cpu()[0]), exact)


def test_consecutive_layout_bit_exact():
    """The consecutive layout (the paper's per-thread loop with the Modified
    Barrett step, serial order restored through LDS): tile sizes from 2 to
    32 outputs per thread, ragged and single-element tails, several tiles
    per workgroup, 16- and 8-byte stores, both kinds."""
    z0 = orc.seed(wl.INDEX_MIN + 4099)
    ref_u, _ = orc.gen(z0, 300_000, "u64", threads=0)
    ref_f, _ = orc.gen(z0, 300_000, "f64", threads=0)
    for block, E, grid in [(256, 0, 0), (64, 2, 3), (128, 32, 5), (512, 8, 0), (1024, 4, 7),
                           (64, 32, 1), (192, 16, 2)]:
        tile = block * (E or 16)
        for count in (1, 2, 17, tile - 1, tile, tile + 1, 3 * tile + 5, 99_991, 300_000):
            if count > 300_000:
                continue
            cfg = nn.make_cfg(block=block, grid=grid, unroll=E, layout="consecutive")
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                for guard in (512, 513):  # 16-byte and 8-byte aligned outputs
                    _say("consecutive", block, E, grid, count, kind, guard)
                    got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=guard)
                    assert np.array_equal(got, ref.view(np.uint64)[:count]), \
                        (block, E, grid, count, kind, guard)
                    assert zn == orc.skip(z0, count)
    cfg = nn.make_cfg(layout="consecutive", temporal=True, width=1)
    got, _ = _gen_guarded(z0, 99_991, "f64", cfg=cfg)
    assert np.array_equal(got, ref_f.view(np.uint64)[:99_991])


def test_consecutive_layout_validation():
    z0 = orc.seed(wl.INDEX_MIN)
    buf = _sentinel_buffer(4097)
    out = buf[:4096].view(torch.float64)
    bad = [nn.make_cfg(layout="consecutive", mulmod="fp64"),
           nn.make_cfg(layout="consecutive", unroll=3),
           nn.make_cfg(layout="consecutive", unroll=64),
           nn.make_cfg(layout="consecutive", ilp=2),
           nn.make_cfg(layout="consecutive", occupancy=3),
           nn.make_cfg(layout="consecutive", block=1024, unroll=32),   # LDS
           nn.make_cfg(layout="consecutive", block=256, unroll=16,
                       grid=(1 << 25) // (256 * 16) + 1),                # skip tables
           nn.make_cfg(mulmod="modbarrett"),                           # rows
           nn.make_cfg(mulmod="modbarrett", layout="flat")]
    for cfg in bad:
        with pytest.raises(nn.NNError):
            nn.generate_into(z0, out, cfg=cfg)
    with pytest.raises(nn.NNError):  # 16-byte stores on an 8-byte aligned output
        nn.generate_into(z0, buf[1:4097].view(torch.float64),
                         cfg=nn.make_cfg(layout="consecutive", width=2))
    with pytest.raises(nn.NNError):
        nn.fill(out, 0, cfg=nn.make_cfg(layout="consecutive"))
    torch.cuda.synchronize()
    assert (_bits(buf) == SENTINEL).all()


def test_counts_beyond_32_bit_indexing():
    """2^33 + 3 raw states (64 GiB) in one call: row pointers, row counts and
    the ragged tail past 2^32 elements; windows sampled against the oracle
    started there by skip-ahead, and the state hand-off."""
    n = (1 << 33) + 3
    z0 = orc.seed(wl.INDEX_MIN + 2024)
    out = torch.empty(n, dtype=torch.uint64, device="cuda")
    zn = nn.generate_into(z0, out)
    torch.cuda.synchronize()
    assert zn == orc.skip(z0, n)
    flat = out.view(torch.int64)
    for st in (0, (1 << 32) - 2048, (1 << 32) + 12345, (1 << 33) - 4096, n - 4096):
        ref, _ = orc.gen(orc.skip(z0, st), 4096, "u64")
        got = flat[st:st + 4096].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), st
    del out, flat
    torch.cuda.empty_cache()


def test_paper_strided_layout_is_the_transposed_sequence():
    """The paper's own layout (Section 3.2), kept for comparison: thread t
    of T = count/E makes elements t*E .. t*E+E-1 and stores its i-th at
    t + i*T; read back transposed it is the serial sequence."""
    z0 = orc.seed(wl.INDEX_MIN + 555)
    ref_u, _ = orc.gen(z0, 1 << 20, "u64", threads=0)
    ref_f, _ = orc.gen(z0, 1 << 20, "f64", threads=0)
    for count, E, block in [(4096, 4096, 512), (1 << 20, 4096, 512), (1 << 20, 16, 64),
                            (3 * 1000, 3, 1024), (999_999, 1, 256), (1 << 20, 2, 128),
                            (65_536 * 7, 7 * 512, 256)]:
        cfg = nn.make_cfg(layout="paper_strided", unroll=E, block=block)
        for kind, ref in (("u64", ref_u), ("f64", ref_f)):
            _say("strided", count, E, block, kind)
            got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=513)
            T = count // E
            serial = got.reshape(E, T).T.reshape(-1)
            assert np.array_equal(serial, ref.view(np.uint64)[:count]), (count, E, block, kind)
            assert zn == orc.skip(z0, count)
    out = torch.empty(4096, dtype=torch.float64, device="cuda")
    for cfg in [nn.make_cfg(layout="paper_strided", unroll=3000),       # does not divide
                nn.make_cfg(layout="paper_strided", unroll=16, grid=4),
                nn.make_cfg(layout="paper_strided", unroll=16, mulmod="fp64"),
                nn.make_cfg(layout="paper_strided", unroll=16, width=2)]:
        with pytest.raises(nn.NNError):
            nn.generate_into(z0, out, cfg=cfg)
