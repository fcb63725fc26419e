"""The autotuner's cache on the CPU: what record() stores and the lookups
read back (the device key is stubbed; no GPU is touched)."""
import json

from paper_1206_1187_amd import tune


def test_record_keeps_best_overall_and_best_row_layout(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "_device_key", lambda: "gfx950/256cu")
    path = str(tmp_path / "tuned.json")
    flat = dict(layout="flat", mulmod="fp64", unroll=4, occupancy=4, temporal=True)
    rows_a = dict(layout="rows", block=256, grid=128, mulmod="fp64", ilp=4, unroll=8)
    rows_b = dict(layout="rows", block=256, grid=160, mulmod="fp64", ilp=2, unroll=4)
    results = sorted([(1.25, rows_a), (1.23, flat), (1.30, rows_b)], key=lambda r: r[0])
    tune.record("plain", "f64", 1 << 30, results, path)
    cache = json.load(open(path))
    assert cache["gfx950/256cu/plain/f64/2^30"]["cfg"] == flat
    assert cache["gfx950/256cu/plain_rows/f64/2^30"]["cfg"] == rows_a
    assert tune.best_plain_cfg("f64", 1 << 30, path) == flat
    assert tune.best_plain_cfg("f64", 1 << 30, path, layout="rows") == rows_a
    # the nearest tuned size bucket of the same form and kind
    assert tune.best_plain_cfg("f64", 1 << 28, path, layout="rows") == rows_a
    assert tune.best_plain_cfg("u64", 1 << 28, path) == {}
    # a batch record has no row-layout entry
    tune.record("batch", "f64", 3 << 30, [(3.4, dict(chunks=True, temporal=True, grid=0))], path)
    assert tune.best_batch_cfg("f64", 3 << 30, path) == dict(chunks=True, temporal=True, grid=0)
    assert "gfx950/256cu/plain_rows/f64/2^31" not in json.load(open(path))


def test_shipped_cache_has_both_plain_entries():
    cache = tune.load_cache()
    for kind, b in (("f64", 30), ("u64", 28)):
        assert cache["gfx950/256cu/plain/%s/2^%d" % (kind, b)]["cfg"]
        assert cache["gfx950/256cu/plain_rows/%s/2^%d" % (kind, b)]["cfg"]["layout"] == "rows"
