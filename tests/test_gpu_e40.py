"""GPU parity of the modulus-3^40 generator (nn_e40_generate_ex) against the
oracle: bit-exact raw states and variates, ragged tails, 8- and 16-byte
aligned outputs, several launch shapes, chained calls, extreme states."""
import sys

import numpy as np
import pytest

import oracle as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1206_1187_amd as nn  # noqa: E402

M = 3 ** 40
SENTINEL = 0xDEADBEEFCAFEF00D


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _bits(t):
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def _gen_guarded(state, count, kind, cfg=None, guard=512):
    dt = torch.float64 if kind == "f64" else torch.uint64
    host = np.full(count + 2 * guard, SENTINEL, dtype=np.uint64)
    buf = torch.from_numpy(host.view(np.int64)).cuda()
    new_state = nn.e40_generate_into(state, buf[guard:guard + count].view(dt), cfg=cfg)
    torch.cuda.synchronize()
    got = _bits(buf)
    assert (got[:guard] == SENTINEL).all(), "write before the output"
    assert (got[guard + count:] == SENTINEL).all(), "write past the output"
    return got[guard:guard + count], new_state


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available()
    nn.init(0)
    yield
    torch.cuda.synchronize()


def test_e40_bit_exact_shapes_and_tails():
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 12345)
    ref_u, _ = orc.e40_gen(z0, 300_000, "u64")
    ref_f, _ = orc.e40_gen(z0, 300_000, "f64")
    shapes = [dict(), dict(layout="rows"),
              dict(block=64, grid=3, ilp=1, unroll=1), dict(block=1024, grid=7, ilp=4, unroll=4),
              dict(block=512, grid=129, ilp=2, unroll=2), dict(block=256, grid=1, ilp=4, unroll=1),
              dict(mulmod="montgomery"), dict(mulmod="montgomery", layout="rows"),
              dict(mulmod="montgomery", block=64, grid=5, ilp=4, unroll=2),
              dict(mulmod="fp64", block=128, grid=33, ilp=1, unroll=4)]
    for kw in shapes:
        cfg = nn.make_cfg(**kw)
        for count in (1, 2, 3, 511, 512, 513, 4097, 99_991, 300_000):
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                for guard in (512, 513):
                    _say("e40", kw, count, kind, guard)
                    got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=guard)
                    assert np.array_equal(got, ref.view(np.uint64)[:count]), (kw, count, kind, guard)
                    assert zn == orc.e40_skip(z0, count)
    got, _ = _gen_guarded(z0, 99_991, "f64", cfg=nn.make_cfg(temporal=True))
    assert np.array_equal(got, ref_f.view(np.uint64)[:99_991])


@pytest.mark.parametrize("mulmod", ["fp64", "montgomery"])
def test_e40_flat_layout_bit_exact(mulmod):
    """The flat layout at modulus 3^40: 2 to 32 rows of 512 outputs per
    chunk, one workgroup per chunk or a smaller grid whose workgroups step
    from chunk to chunk (1, 3 and 7 workgroups), residency caps, both store
    policies, ragged tails around the row and chunk sizes, both kinds."""
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 777)
    ref_u, _ = orc.e40_gen(z0, 300_000, "u64")
    ref_f, _ = orc.e40_gen(z0, 300_000, "f64")
    counts = (1, 2, 3, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 8191, 8193,
              99_991, 300_000)
    for rows, grid, occ, temporal in [(0, 0, 0, None), (2, 0, 3, None), (4, 1, 0, None),
                                      (4, 3, 0, False), (8, 7, 5, True), (16, 0, 0, False),
                                      (16, 2, 2, None), (32, 0, 0, None), (32, 3, 4, True)]:
        cfg = nn.make_cfg(layout="flat", mulmod=mulmod, unroll=rows, grid=grid, occupancy=occ,
                          temporal=temporal)
        for count in counts:
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                _say("e40 flat", mulmod, rows, grid, occ, temporal, count, kind)
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg)
                assert np.array_equal(got, ref.view(np.uint64)[:count]), \
                    (rows, grid, occ, temporal, count, kind)
                assert zn == orc.e40_skip(z0, count)
    # an output that is only 8-byte aligned: its first element alone, the
    # rest 16-byte aligned (the default there too, with the FP64 step)
    for cfg in (nn.make_cfg(layout="flat", mulmod=mulmod), nn.make_cfg(mulmod=mulmod)):
        for count in (1, 2, 3, 4097, 300_000 - 1):
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg, guard=513)
                assert np.array_equal(got, ref.view(np.uint64)[:count]), ("8-aligned", count, kind)
                assert zn == orc.e40_skip(z0, count)


def test_e40_flat_xcd_runs_bit_exact():
    """With one workgroup per chunk the FP64 step's flat layout takes whole
    XCD runs (4,194,304 outputs, at every row count) XCD by XCD, then the
    chunks after the last run from their own base, then the tail: counts
    below, at and past one and two runs, every row count, both kinds,
    against the oracle element by element."""
    run = 8 * 4 * 1024 * 1024 // 8
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 4242)
    top = 2 * run + 512 * 7 + 1
    ref_u, _ = orc.e40_gen(z0, top, "u64")
    ref_f, _ = orc.e40_gen(z0, top, "f64")
    for rows in (2, 4, 8, 16, 32):
        cfg = nn.make_cfg(layout="flat", mulmod="fp64", unroll=rows)
        for count in (run - 1, run, run + 3 * 8192 + 5, top):
            for kind, ref in (("u64", ref_u), ("f64", ref_f)):
                _say("e40 flat xcd runs", rows, count, kind)
                got, zn = _gen_guarded(z0, count, kind, cfg=cfg)
                assert np.array_equal(got, ref.view(np.uint64)[:count]), (rows, count, kind)
                assert zn == orc.e40_skip(z0, count)
    # the default on an output that is only 8-byte aligned and large enough:
    # the flat layout with its first element alone
    for kind, ref in (("u64", ref_u), ("f64", ref_f)):
        got, zn = _gen_guarded(z0, top - 1, kind, guard=513)
        assert np.array_equal(got, ref.view(np.uint64)[:top - 1]), ("default 8-aligned", kind)
        assert zn == orc.e40_skip(z0, top - 1)


def test_e40_flat_beyond_one_launch_sampled():
    """More than 2^30 outputs (several flat launches): windows on both
    sides of every launch boundary and at the tail."""
    n = (1 << 30) + 4099
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 31337)
    out = torch.empty(n, dtype=torch.uint64, device="cuda")
    zn = nn.e40_generate_into(z0, out, cfg=nn.make_cfg(layout="flat"))
    torch.cuda.synchronize()
    assert zn == orc.e40_skip(z0, n)
    flat = out.view(torch.int64)
    for st, k in ((0, 8192), ((1 << 30) - 8192, 8192 + 4099), (123_456_789, 4096)):
        ref, _ = orc.e40_gen(orc.e40_skip(z0, st), k, "u64")
        got = flat[st:st + k].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), st
    del out, flat
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mulmod", ["fp64", "montgomery"])
def test_e40_chained_and_extreme_states(mulmod):
    cfg = nn.make_cfg(mulmod=mulmod)
    B = 3 ** 20
    # states at the ends of the range and with limbs at their ends
    for s in (1, 2, M - 1, M - 2, 2 ** 63 + 1, orc.e40_seed(orc.E40_INDEX_MAX),
              B - 1, B + 1, (B - 1) * B + 1, (B - 1) * B + B - 1):
        if s % 3 == 0:
            continue
        ref, zr = orc.e40_gen(s, 70_001, "u64")
        out = torch.empty(70_001, dtype=torch.uint64, device="cuda")
        z = s
        for lo, hi in ((0, 1), (1, 1000), (1000, 1001), (1001, 70_001)):
            _say("e40 chained", mulmod, s, lo, hi)
            z = nn.e40_generate_into(z, out[lo:hi], cfg=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(out), ref), s
        assert z == zr


@pytest.mark.parametrize("mulmod", ["fp64", "montgomery"])
def test_e40_large_sampled(mulmod):
    """2^26 outputs in the default shape; windows of the output compared
    with the oracle started there by skip-ahead."""
    n = 1 << 26
    z0 = orc.e40_seed(orc.E40_INDEX_MIN + 987654321)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    _say("e40 large", mulmod)
    zn = nn.e40_generate_into(z0, out, cfg=nn.make_cfg(mulmod=mulmod))
    torch.cuda.synchronize()
    assert zn == orc.e40_skip(z0, n)
    flat = out.view(torch.int64)
    rng = np.random.default_rng(40)
    starts = [0, n - 4096] + rng.integers(0, n - 4096, 30).tolist()
    for st in starts:
        ref, _ = orc.e40_gen(orc.e40_skip(z0, int(st)), 4096, "f64")
        got = flat[st:st + 4096].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref.view(np.uint64)), st
    del out, flat


def test_e40_config_validation():
    z0 = orc.e40_seed(orc.E40_INDEX_MIN)
    out = torch.empty(4096, dtype=torch.float64, device="cuda")
    for cfg in [nn.make_cfg(width=1), nn.make_cfg(mulmod="barrett"),
                nn.make_cfg(mulmod="shoup"), nn.make_cfg(layout="flat", unroll=3),
                nn.make_cfg(layout="flat", unroll=64), nn.make_cfg(layout="flat", block=128),
                nn.make_cfg(layout="flat", occupancy=1), nn.make_cfg(layout="flat", ilp=2),
                nn.make_cfg(layout="rows", unroll=8), nn.make_cfg(ilp=3), nn.make_cfg(block=100),
                nn.make_cfg(layout="rows", occupancy=3), nn.make_cfg(grid=1 << 20, block=1024),
                nn.make_cfg(layout="consecutive")]:
        with pytest.raises(nn.NNError):
            nn.e40_generate_into(z0, out, cfg=cfg)
