#!/usr/bin/env python3
"""Benchmark of the alpha_{2,3} generator on one MI355X.

One step is the whole plain path over the bulk workload: seed a starting
index (Eq. 2), generate 2^30 binary64 variates and then 2^28 raw uint64
states from that seed (Eq. 3 with per-thread skip-ahead), with the outputs
resident in HBM.  The JSON line reports whole-job variates/s, the
roofline of the dominant kernel (the f64 generator, flat layout) measured with HIP events
on the launch stream, the paper's "Constant" write ceiling for the same
store pattern (Section 4.2), a comparison of the exact reductions, and the
CPU oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
METRIC = "uniform variates/sec at 1 GPU and % of HBM write BW; batched/served vs plain"
# Profile summary holding the HBM byte counters of the dominant kernel.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_generate_flat_fp64_f64.plain_bulk.md")
# Every source the dominant kernel is compiled from: its counters are void
# once any of them changes.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1206_1187_amd", "csrc", f)
                  for f in ("nn_kernels.hip", "nn_kernels.hpp", "nn_arith.hpp", "nn_device.hpp")]
KERNEL_SOURCES += [os.path.join(ROOT, "include", "nn_device.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _timed_kernel(fn, reps, torch):
    """Average duration (s) of fn() enqueued on the current stream, after one
    untimed call (which takes any one-time set-up, such as a table upload)."""
    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in evs]
    return sum(ms) / len(ms) / 1e3


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile():
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None when the kernel sources changed since
    the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def batched_leg(nn, torch, per_stream=True):
    """Config 4: 10,000 streams (lengths log-uniform in [1, 2^22]) as one
    batched launch replayed from the plan's hipGraph, in the shape
    tune.bench_batch_kw gives (the one the full-size parity test compares),
    against the same streams with one nn_generate launch each on the same
    stream; the other batch kernels for comparison."""
    import numpy as np

    from paper_1206_1187_amd import tune

    states, lengths, offsets = tune.batch_workload()
    total = int(lengths.sum())
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    kw = tune.bench_batch_kw(total)
    res = {"workload": "batched: 10,000 seed indices (numpy default_rng(3)), lengths "
                       "log-uniform in [1, 2^22], f64, windows packed back to back",
           "streams": len(states), "variates": total}
    with nn.BatchPlan("f64", len(states), total, **kw) as plan:
        res["cfg"] = dict(plan.cfg().as_dict(), **{k: v for k, v in kw.items()
                                                  if k in ("interleaved", "chunks")})
        for _ in range(8):  # warm-up: first touch of the output (several launches), first replay
            plan.generate(states, lengths, offsets, out)
        graph_s = _timed_kernel(lambda: plan.generate(states, lengths, offsets, out), 10, torch)
    with nn.BatchPlan("f64", len(states), total, graph=False, **kw) as plan:
        for _ in range(3):
            plan.generate(states, lengths, offsets, out)
        direct_s = _timed_kernel(lambda: plan.generate(states, lengths, offsets, out), 10, torch)
    # every batch kernel at its best measured shape, whichever the benchmark runs
    for name, shape in (("blocked_ms", dict(block=256, grid=128, temporal=True)),
                        ("interleaved_ms", dict(block=256, grid=144, cluster=16,
                                                interleaved=True)),
                        ("chunked_ms", dict(chunks=True))):
        with nn.BatchPlan("f64", len(states), total, mulmod="fp64", **shape) as plan:
            for _ in range(3):
                plan.generate(states, lengths, offsets, out)
            res[name] = _timed_kernel(
                lambda: plan.generate(states, lengths, offsets, out), 10, torch) * 1e3
    res["graph_ms"] = graph_s * 1e3
    res["no_graph_ms"] = direct_s * 1e3
    res["variates_per_s"] = total / graph_s
    res["GBps"] = 8.0 * total / graph_s / 1e9
    res["frac_of_hbm_peak"] = res["GBps"] / (HBM_PEAK_GBPS)
    if not per_stream:
        del out
        torch.cuda.empty_cache()
        return res
    batched_bits = out.view(torch.int64)[:4096].cpu().numpy().copy()
    # one launch per stream, same output, same stream
    views = [(int(s), out[int(o):int(o) + int(n)]) for s, n, o in zip(states, lengths, offsets)]
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for s, v in views:
        nn.generate_into(s, v)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res["per_stream_ms"] = a.elapsed_time(b)
    res["per_stream_wall_ms"] = wall * 1e3
    res["speedup_vs_per_stream"] = res["per_stream_ms"] / res["graph_ms"]
    same = np.array_equal(out.view(torch.int64)[:4096].cpu().numpy(), batched_bits)
    res["outputs_equal_sample"] = bool(same)
    del out
    torch.cuda.empty_cache()
    return res


def served_leg(nn, torch):
    """Config 5: Poisson arrivals at 20k req/s for 10 s, sizes log-uniform in
    [256, 2^24], 1,024 client streams, 64 GB output pool; the served form
    against one nn_generate launch per request on the same trace (both
    arrival loops native), then a load sweep (the trace's first 20,000
    requests replayed 4x to 64x faster)."""
    import numpy as np

    from paper_1206_1187_amd import serve
    from paper_1206_1187_amd import workloads as wl

    tr = wl.served()
    states = np.array([nn.seed(int(a)) for a in tr.stream_indices], dtype=np.uint64)
    pool = 64 << 30
    res = {"workload": "served: numpy default_rng(4), 1,024 streams, Poisson 20k req/s for "
                       "10 s, sizes log-uniform in [256, 2^24] f64, 64 GB pool",
           "requests": int(tr.count.size), "variates": int(tr.count.sum())}
    from paper_1206_1187_amd import tune
    shape = tune.best_batch_cfg("f64", int(tr.count.sum()))
    res["batch_cfg"] = shape
    with serve.Server(states, pool, lanes=2, **shape) as srv:
        res["served"] = serve.replay_served_native(srv, tr, timeout_s=120)
    # Requests up to 2^16 outputs through the persistent device queue.
    with serve.Server(states, pool, lanes=2, device_queue=True, **shape) as srv:
        res["served_device_queue"] = serve.replay_served_native(srv, tr, timeout_s=120)
    res["plain_per_request"] = serve.replay_per_request_native(tr, states, pool // 8,
                                                               timeout_s=120)
    n = 20000
    sweep = []
    for scale in (4, 16, 32, 64):
        with serve.Server(states, pool, lanes=2, **shape) as srv:
            a = serve.replay_served_native(srv, tr, time_scale=scale, timeout_s=120, n=n)
        with serve.Server(states, pool, lanes=2, device_queue=True, **shape) as srv:
            q = serve.replay_served_native(srv, tr, time_scale=scale, timeout_s=120, n=n)
        b = serve.replay_per_request_native(tr, states, pool // 8, time_scale=scale,
                                            timeout_s=120, n=n)
        keys = ("variates_per_s", "p50_ms", "p99_ms")
        sweep.append({"load_x": scale, "served": {k: a[k] for k in keys},
                      "served_device_queue": {k: q[k] for k in keys},
                      "plain": {k: b[k] for k in keys}})
    res["load_sweep_first_20000"] = sweep
    torch.cuda.empty_cache()
    return res


def cpu_baseline(case):
    """The oracle on all host threads over one whole step of the workload,
    streamed through one 2^25-element host buffer; plus one thread on a
    2^24-element prefix."""
    import numpy as np

    import oracle as orc

    chunk = 1 << 25
    threads = orc.max_threads()
    z0 = orc.seed(case.index)
    t0 = time.perf_counter()
    for count, dt in ((case.count_f64, np.float64), (case.count_u64, np.uint64)):
        buf = np.empty(chunk, dtype=dt)
        z = z0
        for _ in range(count // chunk):
            z = orc.gen_into(z, buf, threads=0)
    wall = time.perf_counter() - t0
    total = case.count_f64 + case.count_u64
    one = np.empty(1 << 24, dtype=np.float64)
    t1 = time.perf_counter()
    orc.gen_into(z0, one, threads=1)
    wall1 = time.perf_counter() - t1
    # the paper's own serial CPU loop (Section 3.1's Modified Barrett step,
    # the comparator kept in the oracle), one thread, the same prefix
    t2 = time.perf_counter()
    orc.gen_f64_modbarrett(z0, one.size)
    wall2 = time.perf_counter() - t2
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": total / wall,
        "unit": "variates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "one full step (2^30 f64 + 2^28 u64 from the same seed index) in 2^25-element "
                  "chunks, OpenMP skip-ahead partition over %d threads; %.2f s wall" % (threads, wall),
        "single_thread_value": float(one.size / wall1),
        "single_thread_modified_barrett_value": float(one.size / wall2),
        "cpu_model": model,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the fill ceiling and reduction comparison")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form replay")
    ap.add_argument("--no-per-stream", action="store_true",
                    help="skip the batched leg's one-launch-per-stream baseline (10,000 launches; "
                         "for the hardware-counter runs)")
    ap.add_argument("--only", choices=["batched", "served"],
                    help="run only this leg and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (torch) five times, "
                         "to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU only: this program has no multi-GPU path "
            "(--gpus %d requested)." % args.gpus)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        log("bench.py runs as a single process on one GPU.")
        sys.exit(2)

    import torch

    import paper_1206_1187_amd as nn
    from paper_1206_1187_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 5 x %d bytes" % (src.numel() * 8))
        return
    nn.init(0)
    if args.only:
        leg = (batched_leg(nn, torch, not args.no_per_stream) if args.only == "batched"
               else served_leg(nn, torch))
        print(json.dumps({args.only: leg}), flush=True)
        return
    case = wl.plain_bulk()
    out_f = torch.empty(case.count_f64, dtype=torch.float64, device="cuda")
    out_u = torch.empty(case.count_u64, dtype=torch.uint64, device="cuda")
    # Both kinds in the launch configuration tune.BENCH_PLAIN names (the
    # flat layout: chunks of four 512-output rows per workgroup, temporal
    # stores, residency cap 4), the one the full-size parity tests compare.
    from paper_1206_1187_amd import tune
    cfg_f = tune.bench_plain_cfg("f64")
    cfg_u = tune.bench_plain_cfg("u64")
    # the row layout in its tuned shape, for comparison
    cfg_rows_f = nn.make_cfg(**dict(tune.best_plain_cfg("f64", case.count_f64, layout="rows"),
                                    layout="rows"))
    cfg_rows_u = nn.make_cfg(**dict(tune.best_plain_cfg("u64", case.count_u64, layout="rows"),
                                    layout="rows"))
    log("workload", case, "cfg f64", cfg_f.as_dict(), "cfg u64", cfg_u.as_dict())

    def step(ev=None):
        s = nn.seed(case.index)
        if ev is not None:
            ev[0].record()
        nn.generate_into(s, out_f, cfg=cfg_f)
        if ev is not None:
            ev[1].record()
        nn.generate_into(s, out_u, cfg=cfg_u)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    f64_ms = [a.elapsed_time(b) for a, b in evs]
    f64_s = sum(f64_ms) / len(f64_ms) / 1e3
    per_step = case.count_f64 + case.count_u64
    value = per_step * args.steps / elapsed
    achieved = 8.0 * case.count_f64 / f64_s / 1e9
    log("timed %d steps in %.3f s: %.4g variates/s; f64 kernel %.3f ms = %.1f GB/s"
        % (args.steps, elapsed, value, f64_s * 1e3, achieved))

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "variates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain bulk: seed index %d (numpy default_rng(1) over [3^33+100, 2^53]), "
                        "2^30 f64 variates then 2^28 u64 states per step" % case.index,
            "count_f64": case.count_f64,
            "count_u64": case.count_u64,
            "launch_f64": cfg_f.as_dict(),
            "launch_u64": cfg_u.as_dict(),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic_from_profile(),
            "kernel": "k_generate_flat<VarFP64, 1, false, 4, 256> (f64, flat: 4 rows of 512 per "
                      "workgroup in XCD runs of 256 chunks, temporal stores, residency cap 4)",
            "algorithmic_bytes_per_launch": 8 * case.count_f64,
        },
    }

    if not args.no_extras:
        extras = {}
        reps = 20
        u_s = _timed_kernel(lambda: nn.generate_into(nn.seed(case.index), out_u, cfg=cfg_u), reps,
                            torch)
        extras["generate_u64_GBps"] = 8.0 * case.count_u64 / u_s / 1e9
        # nn_generate with no configuration (the library's default layout)
        for kind, out in (("f64", out_f), ("u64", out_u)):
            d_s = _timed_kernel(lambda: nn.generate_into(nn.seed(case.index), out), reps, torch)
            extras["library_default_%s_GBps" % kind] = 8.0 * out.numel() / d_s / 1e9
        # the row layout (tuned shape) for both kinds
        rows_s = _timed_kernel(lambda: nn.generate_into(nn.seed(case.index), out_f,
                                                        cfg=cfg_rows_f), reps, torch)
        extras["rows_layout_f64_GBps"] = 8.0 * case.count_f64 / rows_s / 1e9
        rows_u_s = _timed_kernel(lambda: nn.generate_into(nn.seed(case.index), out_u,
                                                          cfg=cfg_rows_u), reps, torch)
        extras["rows_layout_u64_GBps"] = 8.0 * case.count_u64 / rows_u_s / 1e9
        # the flat layout's XCD runs against its chunks in address order
        # (NN_CFG_ADDRESS_ORDER), the benchmark's own launches otherwise,
        # timed in turn over three rounds (best round each)
        order = {}
        for kind, out, cfg in (("f64", out_f, cfg_f), ("u64", out_u, cfg_u)):
            addr = nn._native.LaunchCfg.from_buffer_copy(cfg)
            addr.flags |= nn._native.NN_CFG_ADDRESS_ORDER
            best = {}
            for _ in range(3):
                for name, c in (("xcd_runs", cfg), ("address_order", addr)):
                    t = _timed_kernel(lambda: nn.generate_into(nn.seed(case.index), out, cfg=c),
                                      reps, torch)
                    best[name] = min(best.get(name, t), t)
            order[kind] = {k + "_GBps": 8.0 * out.numel() / v / 1e9 for k, v in best.items()}
        extras["flat_chunk_order"] = order
        # The paper's "Constant" kernel (Section 4.2, Tables 1-2): the f64
        # generator's own launch (same layout, rows, store policy and cap)
        # with the arithmetic taken out -- bare stores, and the same stores
        # after the generator's start-up table loads (the generator minus its
        # arithmetic); the row layout's pattern; and the fastest fill pattern
        # measured (one row per workgroup, cap 3).
        value = 0x3FE0000000000000
        fills = {"fill_same_pattern": (cfg_f, False), "fill_same_pattern_with_start": (cfg_f, True),
                 "fill_row_pattern": (cfg_rows_f, False),
                 "fill_one_row_cap3": (nn.make_cfg(layout="flat", unroll=1, occupancy=3,
                                                   temporal=True), False)}
        fill_s = {}
        for name, (cfg, start) in fills.items():
            fill_s[name] = _timed_kernel(lambda: nn.fill(out_f, value, cfg=cfg, with_start=start),
                                         reps, torch)
            extras[name + "_GBps"] = 8.0 * case.count_f64 / fill_s[name] / 1e9
        best = min(fill_s.values())
        extras["write_ceiling_GBps"] = 8.0 * case.count_f64 / best / 1e9
        extras["f64_frac_of_write_ceiling"] = achieved / extras["write_ceiling_GBps"]
        # Paper's Table 2: generation time net of the memory-access time,
        # against the generator minus its arithmetic (the same pattern after
        # the same start-up loads), against the bare same-pattern fill
        # (negative when the stores paced by the arithmetic write faster than
        # the same stores back to back) and against the fastest fill.
        extras["net_generation_ms"] = (f64_s - fill_s["fill_same_pattern_with_start"]) * 1e3
        extras["net_generation_same_pattern_ms"] = (f64_s - fill_s["fill_same_pattern"]) * 1e3
        extras["net_generation_vs_fastest_fill_ms"] = (f64_s - best) * 1e3
        # Paper's Table 1, execution vs including setup: the host seeding of
        # Eq. 2 (a 106-bit power modulo 3^33 from the index), the launch
        # constants and the launch, then the kernel, timed on the host clock
        # from the index to the synchronised result.
        t_seed = time.perf_counter()
        for _ in range(10000):
            nn.seed(case.index)
        extras["seed_host_us"] = (time.perf_counter() - t_seed) / 10000 * 1e6
        walls = []
        for _ in range(10):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nn.generate_into(nn.seed(case.index), out_f, cfg=cfg_f)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        extras["f64_kernel_ms"] = f64_s * 1e3
        extras["f64_including_setup_ms"] = sorted(walls)[len(walls) // 2] * 1e3
        # Fused consumer: the same generation summed in registers (no stores),
        # the analogue of the paper's Table 2 net generation rate.
        res = torch.zeros(1, dtype=torch.int64, device="cuda")
        cons_s = _timed_kernel(lambda: nn.consume(nn.seed(case.index), case.count_f64, "u64",
                                                  result=res), reps, torch)
        resf = torch.zeros(1, dtype=torch.float64, device="cuda")
        consf_s = _timed_kernel(lambda: nn.consume(nn.seed(case.index), case.count_f64, "f64",
                                                   result=resf), reps, torch)
        extras["fused_consumer_u64_variates_per_s"] = case.count_f64 / cons_s
        extras["fused_consumer_f64_variates_per_s"] = case.count_f64 / consf_s
        shoot = {}
        for name in ("fp64", "barrett", "shoup", "montgomery"):
            for kind, out in (("f64", out_f), ("u64", out_u)):
                cfg = nn.make_cfg(mulmod=name)
                s = _timed_kernel(
                    lambda: nn.generate_into(nn.seed(case.index), out, cfg=cfg), 10, torch)
                shoot["%s_%s_GBps" % (name, kind)] = 8.0 * out.numel() / s / 1e9
        # The paper's own step (Section 3.1's Modified Barrett by 2^53) in
        # its per-thread consecutive loop, serial order kept through LDS.
        for kind, out in (("f64", out_f), ("u64", out_u)):
            cfg = nn.make_cfg(layout="consecutive")
            s = _timed_kernel(
                lambda: nn.generate_into(nn.seed(case.index), out, cfg=cfg), 10, torch)
            shoot["modbarrett_consecutive_%s_GBps" % kind] = 8.0 * out.numel() / s / 1e9
            # ... and in the paper's own transposed layout (512 threads x 4096).
            cfg = nn.make_cfg(layout="paper_strided")
            s = _timed_kernel(
                lambda: nn.generate_into(nn.seed(case.index), out, cfg=cfg), 10, torch)
            shoot["modbarrett_paper_strided_%s_GBps" % kind] = 8.0 * out.numel() / s / 1e9
        extras["mulmod_shootout_default_shape"] = shoot
        # Section 2's larger modulus 3^40: the library default (FP64 step on
        # base-3^20 limbs, the flat layout with 16 rows per chunk in XCD runs),
        # the flat layout with 8 rows, the row layout and the Montgomery step.
        # Every configuration is run once before any is timed, then the
        # configurations are timed in turn over four rounds, in reverse order
        # every other round (the best round counts): the first few dozen 3^40
        # launches of a process ran several per cent slower than later ones
        # of the same kernel.
        z40 = nn.e40_seed(nn.E40_INDEX_MIN)
        for kind, out in (("f64", out_f), ("u64", out_u)):
            e40_cfgs = (("", None), ("_flat", nn.make_cfg(layout="flat", unroll=8)),
                        ("_rows", nn.make_cfg(layout="rows")),
                        ("_montgomery", nn.make_cfg(mulmod="montgomery")))
            for _, cfg in e40_cfgs:
                nn.e40_generate_into(z40, out, cfg=cfg)
            best = {}
            for rnd in range(4):
                for name, cfg in (e40_cfgs if rnd % 2 == 0 else e40_cfgs[::-1]):
                    s = _timed_kernel(lambda: nn.e40_generate_into(z40, out, cfg=cfg), 10, torch)
                    best[name] = min(best.get(name, s), s)
            for name, s in best.items():
                extras["modulus_3e40%s_%s_GBps" % (name, kind)] = 8.0 * out.numel() / s / 1e9
        result["extras"] = extras
        log("extras", json.dumps(extras))

    del out_f, out_u
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["batched"] = batched_leg(nn, torch, not args.no_per_stream)
        log("batched", json.dumps(result["batched"]))
        if not args.no_served:
            result["served"] = served_leg(nn, torch)
            log("served", json.dumps(result["served"]))
    if not args.no_cpu_baseline:
        cb = cpu_baseline(case)
        log("cpu_baseline", json.dumps(cb))
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
