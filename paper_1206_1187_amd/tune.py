"""Autotuner for the launch shapes of the plain and batched forms.

Times candidate configurations on a workload with HIP events (median of
repeated launches) and records the fastest in a JSON cache keyed by device
architecture, compute-unit count, form, output kind and a size bucket.  The
binding reads the cache through ``best_plain_cfg`` / ``best_batch_cfg``.

    python -m paper_1206_1187_amd.tune --form batch --kind f64
    python -m paper_1206_1187_amd.tune --form plain --kind u64
"""
import argparse
import itertools
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")


def _device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s/%dcu" % (arch, p.multi_processor_count)


def _bucket(n):
    return "2^%d" % max(0, int(math.floor(math.log2(max(1, int(n))))))


def _key(form, kind, size):
    return "%s/%s/%s/%s" % (_device_key(), form, kind, _bucket(size))


def load_cache(path=CACHE):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _lookup(form, kind, size, path=CACHE):
    cache = load_cache(path)
    entry = cache.get(_key(form, kind, size))
    if entry is None:
        # nearest tuned bucket of the same device, form and kind
        prefix = "%s/%s/%s/" % (_device_key(), form, kind)
        best = None
        for k, v in cache.items():
            if k.startswith(prefix):
                d = abs(int(k.rsplit("^", 1)[1]) - int(_bucket(size)[2:]))
                if best is None or d < best[0]:
                    best = (d, v)
        entry = best[1] if best else None
    return dict(entry["cfg"]) if entry else {}


#: The launch configurations bench.py times on the plain bulk workload, by
#: output kind (make_cfg keyword arguments).  The full-size GPU parity tests
#: run exactly these, so the timed kernels are the compared ones.
BENCH_PLAIN = {
    "f64": dict(layout="flat", mulmod="fp64", unroll=4, occupancy=4, temporal=True),
    # raw states: the FP64 reduction too (the library default and the
    # autotuner's pick with the chunks in XCD runs; Shoup's, which keeps the
    # state an integer, ties or trails by 1-2 % there)
    "u64": dict(layout="flat", mulmod="fp64", unroll=4, occupancy=4, temporal=True),
}


def bench_plain_cfg(kind):
    """nn_launch_cfg of the benchmark's plain-bulk launch for `kind` ("f64"
    or "u64")."""
    import paper_1206_1187_amd as nn
    return nn.make_cfg(**BENCH_PLAIN[kind])


def bench_batch_kw(total, path=CACHE):
    """BatchPlan keyword arguments of the benchmark's batched leg (f64,
    `total` outputs): the tuned shape."""
    return best_batch_cfg("f64", total, path)


def best_plain_cfg(kind, count, path=CACHE, layout=None):
    """make_cfg keyword arguments tuned for ``count`` outputs, or {};
    ``layout="rows"``: the best shape of the row layout."""
    return _lookup("plain" if layout is None else "plain_" + layout, kind, count, path)


def best_batch_cfg(kind, total, path=CACHE):
    """BatchPlan keyword arguments tuned for ``total`` outputs, or {}."""
    return _lookup("batch", kind, total, path)


def _median_ms(fn, reps, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    return ms[len(ms) // 2]


def _min_ms(fn, reps, rounds):
    """Best over `rounds` of the mean duration of `reps` launches of fn()
    (one untimed launch before each round), in ms."""
    import torch
    best = float("inf")
    for _ in range(rounds):
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        best = min(best, sum(a.elapsed_time(b) for a, b in evs) / reps)
    return best


def pick_plain_grid(cfg, out, state, deltas, rounds=3, reps=5):
    """The launch shape `cfg` (an nn_launch_cfg) with the grid that runs
    fastest on the current device among cfg.grid + d, d in `deltas`: the best
    grid of a tuned shape differs between MI355X GPUs by about one such
    step.  Times generate_into(state, out) for each candidate, interleaving
    the candidates over `rounds` rounds.  Returns (cfg, {grid: ms})."""
    import paper_1206_1187_amd as nn
    cands = []
    for d in deltas:
        c = type(cfg)(*[getattr(cfg, f) for f, _ in cfg._fields_])
        c.grid = max(16, cfg.grid + d)
        cands.append(c)
    times = {c.grid: float("inf") for c in cands}
    for _ in range(rounds):
        for c in cands:
            times[c.grid] = min(times[c.grid],
                                _min_ms(lambda: nn.generate_into(state, out, cfg=c), reps, 1))
    return min(cands, key=lambda c: times[c.grid]), times


def pick_plain_layout(cfg, out, state, rounds=3, reps=5):
    """`cfg` (a row-layout nn_launch_cfg, NN_CFG_ROWS set) or the flat layout
    at its library defaults (fields 0: four 512-output rows per workgroup,
    temporal stores, residency cap 4), whichever runs faster on the current
    device (on an output that is only 8-byte aligned the flat layout writes
    its first element alone).  Returns (cfg, {"rows": ms, "flat": ms})."""
    import paper_1206_1187_amd as nn
    flat = nn.make_cfg(layout="flat", mulmod=int(cfg.mulmod))
    cands = {"rows": cfg, "flat": flat}
    times = {k: float("inf") for k in cands}
    for _ in range(rounds):
        for k, c in cands.items():
            times[k] = min(times[k], _min_ms(lambda: nn.generate_into(state, out, cfg=c), reps, 1))
    return cands[min(times, key=times.get)], times


def pick_batch_grid(kw, kind, states, lengths, offsets, out, rounds=2, reps=3):
    """BatchPlan keyword arguments `kw` with the grid (or a neighbour one
    cluster away, the cluster kept) that replays fastest on the current
    device.  Returns (kw, {grid: ms}, {grid: plan}); the caller owns the
    candidates' plans and closes them (reusing the chosen one avoids freeing
    and allocating workspaces just before its own measurement)."""
    import paper_1206_1187_amd as nn
    if not kw.get("grid"):
        return dict(kw), {}, {}
    step = max(16, int(kw.get("cluster") or 16))
    grids = [g for g in (kw["grid"], kw["grid"] - step, kw["grid"] + step)
             if g > 0 and not (kw.get("cluster") and g % kw["cluster"])]
    total = int(sum(int(n) for n in lengths))
    plans = {}
    try:
        for g in grids:
            plans[g] = nn.BatchPlan(kind, len(states), total, **dict(kw, grid=g))
        times = {}
        for _ in range(rounds):
            for g in grids:
                times[g] = min(times.get(g, float("inf")), _min_ms(
                    lambda: plans[g].generate(states, lengths, offsets, out), reps, 1))
    except BaseException:
        for p in plans.values():
            p.close()
        raise
    return dict(kw, grid=min(times, key=times.get)), times, plans


def tune_plain(kind, count, reps=9, log=print):
    import torch

    import paper_1206_1187_amd as nn
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    dt = torch.float64 if kind == "f64" else torch.uint64
    out = torch.empty(count, dtype=dt, device="cuda")
    s0 = nn.seed(nn.INDEX_MIN)
    results = []
    grids = sorted({max(1, cus * k // 8) for k in (2, 3, 4, 5, 6, 8)})
    cands = [dict(block=256, grid=grid, mulmod=mulmod, ilp=ilp, unroll=unroll, width=2,
                  layout="rows", temporal=temporal)
             for mulmod, grid, ilp, unroll, temporal in itertools.product(
                 ("fp64", "shoup"), grids, (1, 2, 4), (2, 4, 8), (False, True))]
    # flat layout: `unroll` rows of 512 outputs per workgroup, one workgroup
    # per chunk, residency capped at `occupancy` workgroups per compute unit
    cands += [dict(layout="flat", mulmod=mulmod, unroll=rows, occupancy=occ, temporal=temporal)
              for mulmod, rows, occ, temporal in itertools.product(
                  ("fp64", "shoup"), (2, 4, 8), (3, 4, 5, 6), (False, True))]
    # four-row chunks in address order instead of XCD runs
    cands += [dict(layout="flat", mulmod=mulmod, unroll=4, occupancy=occ, temporal=True,
                   address_order=True)
              for mulmod, occ in itertools.product(("fp64", "shoup"), (3, 4, 5))]
    for kw in cands:
        cfg = nn.make_cfg(**kw)
        ms = _median_ms(lambda: nn.generate_into(s0, out, cfg=cfg), reps)
        results.append((ms, kw))
        log(json.dumps(dict(kw, ms=ms, GBps=8 * count / ms / 1e6)))
    results.sort(key=lambda r: r[0])
    return results


def batch_workload():
    """The batched workload: 10,000 streams, lengths log-uniform in [1, 2^22]."""
    import numpy as np

    import paper_1206_1187_amd as nn
    from paper_1206_1187_amd import workloads as wl
    case = wl.batched()
    states = np.array([nn.seed(int(a)) for a in case.indices], dtype=np.uint64)
    lengths = case.lengths
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.uint64)
    return states, lengths, offsets


def tune_batch(kind, reps=5, log=print, workload=None):
    import torch

    import paper_1206_1187_amd as nn
    states, lengths, offsets = workload if workload is not None else batch_workload()
    total = int(lengths.sum())
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    dt = torch.float64 if kind == "f64" else torch.uint64
    out = torch.empty(total, dtype=dt, device="cuda")
    results = []
    grids = sorted({max(1, cus * k // 16) for k in (4, 6, 8, 9, 10, 12, 16, 24, 32)})
    shapes = [dict(mulmod=m, block=b, cluster=k, temporal=t) for m in ("fp64", "shoup")
              for b in (256, 512) for k in (1, 4, 8, 16) for t in (False, True)]
    shapes += [dict(mulmod=m, block=256, cluster=8) for m in ("barrett", "montgomery")]
    # interleaved kernel: cluster 0 = all workgroups interleave over one range
    shapes += [dict(mulmod="fp64", block=256, cluster=k, temporal=t, interleaved=True)
               for k in (0, 8, 16, 32) for t in (False, True)]
    cands = [dict(shape, grid=grid) for shape, grid in itertools.product(shapes, grids)
             if not (shape["cluster"] and grid % shape["cluster"])]
    # chunked kernel: one workgroup per 16 KiB chunk (grid 0) at residency
    # caps around the plain flat layout's, or persistent
    cands += [dict(mulmod="fp64", chunks=True, temporal=t, grid=0, occupancy=o)
              for t in (False, True) for o in (3, 4, 5, 6, 8)]
    cands += [dict(mulmod="fp64", chunks=True, temporal=t, grid=g)
              for t in (False, True) for g in (cus * 2, cus * 4)]
    for kw in cands:
        with nn.BatchPlan(kind, len(states), total, **kw) as plan:
            ms = _median_ms(lambda: plan.generate(states, lengths, offsets, out), reps)
        results.append((ms, kw))
        log(json.dumps(dict(kw, ms=ms, GBps=8 * total / ms / 1e6)))
    results.sort(key=lambda r: r[0])
    return results


def record(form, kind, size, results, path=CACHE):
    """Records the fastest of `results` (sorted (ms, kw) pairs) for `form`;
    for the plain form also the fastest row-layout shape (form "plain_rows"),
    which callers that run the row kernel on purpose read."""
    cache = load_cache(path)
    entries = [(form, results)]
    if form == "plain":
        entries.append(("plain_rows", [r for r in results if r[1].get("layout") == "rows"]))
    for f, res in entries:
        if not res:
            continue
        ms, kw = res[0]
        cache[_key(f, kind, size)] = {
            "cfg": kw,
            "ms": ms,
            "GBps": 8 * size / ms / 1e6,
            "candidates": len(res),
            "tuned_at": time.strftime("%Y-%m-%d"),
        }
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return cache


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--form", choices=["plain", "batch"], required=True)
    ap.add_argument("--kind", choices=["f64", "u64"], default="f64")
    ap.add_argument("--count", type=int, default=1 << 30, help="plain form: outputs per launch")
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args(argv)
    import torch

    import paper_1206_1187_amd as nn
    torch.cuda.set_device(0)
    nn.init(0)

    def log(line):
        print(line, file=sys.stderr, flush=True)

    if args.form == "plain":
        res = tune_plain(args.kind, args.count, log=log)
        size = args.count
    else:
        wk = batch_workload()
        res = tune_batch(args.kind, log=log, workload=wk)
        size = int(wk[1].sum())
    record(args.form, args.kind, size, res, args.cache)
    print(json.dumps({"form": args.form, "kind": args.kind, "best": res[0][1],
                      "ms": res[0][0], "GBps": 8 * size / res[0][0] / 1e6}), flush=True)


if __name__ == "__main__":
    main()
