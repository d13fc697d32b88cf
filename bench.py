#!/usr/bin/env python3
"""Throughput of the P_l + B_l hot path on one MI355X.

Workload (one "step"): a batch of 64 synthetic lognormal mock catalogs of
uneven size (N_g log-uniform in [1e6, 8e6], 10x randoms), 256^3 TSC mesh with
interlacing, L = 1000 Mpc/h, observer 1500 Mpc/h from the box corner; per mock
the Yamamoto P_0, P_2, P_4 and the Scoccimarro B_0 (20 bins of dk = 0.01,
825 closed triangles) with analytic shot noise.  Catalogs are resident in HBM
before timing.  Prints one JSON line.

Also measured: the plain FP64 GPU path (same algorithm, FP64 fields and
contraction) on a few mocks, per-kernel HIP-event timings of the dominant
kernel for the roofline, and the FP64 CPU oracle on a bounded sample.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import ctypes as C
import json
import math
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")  # the CPU oracle runs single-threaded

import numpy as np

HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mocks", type=int, default=64)
    ap.add_argument("--precision", choices=["f32", "bf16x3"], default="bf16x3")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of one hipGraph")
    ap.add_argument("--graph-per-stream", action="store_true",
                    help="one single-stream graph per stream instead of one multi-stream graph")
    ap.add_argument("--streams", type=int, default=0,
                    help="concurrent streams inside a step (0: the autotuner's choice, else 4)")
    ap.add_argument("--engine", choices=["native", "torch"], default="native",
                    help="batch runner: the library's cnpc_batch (HIP graph captured by the library) "
                         "or the Python Batch captured with torch.cuda.CUDAGraph")
    ap.add_argument("--no-tune", action="store_true", help="library defaults, no autotuning")
    ap.add_argument("--balance", choices=["rr", "lpt", "mixed"], default="rr",
                    help="placement of the catalogs on the streams (see pipeline.Batch.assignment)")
    ap.add_argument("--tune-mocks", type=int, default=16, help="mocks per autotuner trial batch")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--fp64-mocks", type=int, default=2, help="mocks timed on the plain FP64 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-core oracle sample (0: min(cpu count, 16))")
    ap.add_argument("--cpu-whole", action="store_true",
                    help="only time the oracle on whole mocks (CPU only; takes about an hour)")
    ap.add_argument("--cpu-sample-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4, 5],
                    help="4: the batched headline; 1, 2, 3, 5: one catalog of that configuration "
                         "timed per precision form, with cross-precision errors")
    ap.add_argument("--reps", type=int, default=2, help="timed repetitions per form (--config != 4)")
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def make_mocks(nmocks: int, workers: int = 16):
    import synthcat
    sizes = synthcat.mock_sizes_c4(64)[:nmocks]

    def one(k):
        ng = int(sizes[k])
        g = synthcat.lognormal_catalog(ng, 1000.0, 4000 + 2 * k)
        r = synthcat.random_catalog(10 * ng, 4000 + 2 * k + 1)
        return g, r

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(nmocks))), sizes


def pipeline_bytes(ng, nr, es=4, n=256):
    """Minimal HBM bytes of one mock when every stage reads its inputs and
    writes its outputs once: 12 (N_g + N_r) + 50 R + 34 C (R: real mesh, C:
    half-complex spectrum)."""
    R = n ** 3 * es
    Cb = n * n * (n // 2 + 1) * 2 * es
    return 12 * (ng + nr) + 50 * R + 34 * Cb


def stage_model(ng, nr, n=256, es=4, grid=128, rows=110, cols=20):
    """Algorithmic HBM bytes of one mock per stage of the byte model (every
    stage reads its inputs and writes its outputs once; R: real mesh, C:
    half-complex spectrum) and the contraction's MFMA flops.  The stages sum to
    pipeline_bytes: paint 12 (N_g + N_r) + 4R; the transforms 26R + 18C
    (interlaced r2c x4 4R + 2C, de-alias c2r C + R, Y_lm r2c x14 R + 14C, 20
    shell c2r C + 20R); binning 16C; contraction 20R.  MFMA flops: the 32 x 32
    output tiles over the contraction's pair rows and columns, three split
    products, 2 flops per multiply-add, over the grid^3 points."""
    R = n ** 3 * es
    Cb = n * n * (n // 2 + 1) * 2 * es
    tiles = -(-rows // 32) * 32 * -(-cols // 32) * 32
    return {"paint": 12 * (ng + nr) + 4 * R, "fft": 26 * R + 18 * Cb, "bin": 16 * Cb,
            "contract": 20 * R, "contract_flops": 3 * 2.0 * tiles * grid ** 3}


# kernel-timer classes behind each stage of the byte model; sums and sort are
# intermediates of this design (the particle reads are counted once, in paint)
STAGE_CLASSES = {"paint": ("paint",), "fft": ("fold", "zr2c", "col", "zc2r"), "bin": ("bin",),
                 "contract": ("contract",), "intermediate": ("sums", "sort")}


def copy_probe(mib: int):
    """A plain copy kernel of known size (5 launches): under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE per dispatch calibrate the counters against bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 5}))


def copy_rate_gbs(mib: int = 2048, reps: int = 10) -> float:
    """Achievable HBM rate of a plain streaming copy, b = 1 * a through torch's
    elementwise kernel (6.1-6.2 TB/s on MI355X, where its blit copy b.copy_(a)
    reaches 4.3-5.0), on arrays far larger than the 256 MB last-level cache:
    bytes read plus written per second, median of `reps` copies timed with HIP
    events."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        torch.mul(a, 1.0, out=b)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))
    del a, b
    return 2.0 * n * 4 / (ms / 1e3) / 1e9


def main():
    args = parse()
    if args.cpu_sample_worker:
        _sample_worker(args.cpu_sample_worker)
        return
    if args.cpu_whole:
        cpu_whole(args)
        return
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; the mocks are independent and "
                          "would shard across GPUs without communication, but no multi-GPU "
                          "path is implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.config != 4:
        single_config(args)
        return
    import torch
    import paper_2605_04864_amd as cn
    from paper_2605_04864_amd import _lib as L
    from paper_2605_04864_amd import pipeline as pl
    import synthcat

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    mocks, sizes = make_mocks(args.mocks)
    log(args, f"generated {args.mocks} mocks in {time.time() - t0:.1f}s")
    t_up = time.perf_counter()
    gpu_mocks = [(torch.from_numpy(g).to(dev), torch.from_numpy(r).to(dev)) for g, r in mocks]
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t_up
    up_bytes = float(sum(g.nbytes + r.nbytes for g, r in mocks))
    log(args, f"uploaded in {time.time() - t0:.1f}s")
    obs = synthcat.observer_position()
    bins = cn.kbins(0.0, 0.01, 20)
    prec = L.PREC_BF16X3 if args.precision == "bf16x3" else L.PREC_F32
    desc = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=obs)
    sc = pl.Scratch()
    t_plan = time.perf_counter()
    plan = pl.bispec_plan(desc, bins, L.EST_SCOCCIMARRO, 0, prec, sc)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t_plan
    outs = [{"pk": torch.empty((9, 20), dtype=torch.float64, device=dev),
             "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device=dev)} for _ in gpu_mocks]
    tuning = None
    nstreams = args.streams or 4
    if not args.no_tune:
        from paper_2605_04864_amd import autotune
        tcat = gpu_mocks[: max(1, min(args.tune_mocks, len(gpu_mocks)))]
        res = autotune.tune_batch(desc, tcat, bins, plan, use_cache=False, reps=5,
                                  streams=(args.streams,) if args.streams else (1, 2, 3, 4, 6),
                                  log=lambda m: log(args, m), engine=args.engine)
        nstreams = res.streams
        tuning = res.as_dict()
        tuning["batch_mocks"] = len(tcat)
        log(args, f"autotuned in {res.seconds:.1f}s: streams {res.streams}, knobs {res.knobs}, "
                  f"{res.default_ms:.2f} -> {res.ms:.2f} ms per {len(tcat)} mocks")
    native = args.engine == "native" and not args.graph_per_stream and args.balance == "rr"
    if native:
        batch = pl.NativeBatch(desc, bins, plan, nstreams=nstreams,
                               max_ngal=max(int(g.shape[1]) for g, _ in gpu_mocks),
                               max_nran=max(int(r.shape[1]) for _, r in gpu_mocks))

        def step():
            batch.run(gpu_mocks, outs)
    else:
        batch = pl.Batch(nstreams, balance=args.balance)

        def step():
            batch.run(desc, gpu_mocks, bins, plan, outs)

    t_eager = time.perf_counter()
    step()  # eager pass: plans, twiddles and scratch reach their final size
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t_eager
    eager = [(o["pk"].clone(), o["bk"].clone()) for o in outs]
    vs_oracle = smallest_mock_vs_oracle(mocks, sizes, eager, args.mocks)

    ntot = int(np.sum(sizes[: args.mocks]) * 11)
    # contraction rows: the shell pairs (j, k) of the kept configurations
    rows = len({(int(c[1]), int(c[2])) for c in plan.configs()[0]})
    models = [stage_model(int(sz), 10 * int(sz), grid=plan.grid, rows=rows) for sz in sizes[: args.mocks]]
    model = {k: float(np.sum([m[k] for m in models])) for k in models[0]}  # per step

    run = step
    t_cap = None
    if args.graph_per_stream and not args.no_graph:
        # one single-stream graph per stream, replayed side by side
        graphs = []
        for k, s in enumerate(batch.streams):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                batch.run_stream(k, desc, gpu_mocks, bins, plan, outs)
            graphs.append(g)

        def run():
            cur = torch.cuda.current_stream()
            for s in batch.streams:
                s.wait_stream(cur)
            for g, s in zip(graphs, batch.streams):
                with torch.cuda.stream(s):
                    g.replay()
            for s in batch.streams:
                cur.wait_stream(s)
        log(args, f"captured {len(graphs)} single-stream graphs")
    elif not args.no_graph and native:
        t_cap = time.perf_counter()
        batch.capture(gpu_mocks, outs)
        torch.cuda.synchronize()
        t_cap = time.perf_counter() - t_cap
        run = batch.replay
        log(args, "captured the batch as one graph (cnpc_batch_capture)")
    elif not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
        log(args, "captured the batch as one graph")
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    log(args, f"warmup done {time.time() - t0:.1f}s")
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        run()
        evs[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    # the timed replays recompute every output: they must match the eager pass
    replay_err = 0.0
    for (pk, bk), o in zip(eager, outs):
        for a, b in ((o["pk"], pk), (o["bk"], bk)):
            replay_err = max(replay_err, float((a - b).abs().max() / b.abs().max().clamp_min(1e-300)))
    del eager
    value = args.mocks / (ms_step / 1e3)
    log(args, f"timed {args.steps} steps: {ms_step:.1f} ms/step (wall {wall:.2f}s)")

    # plain FP64 GPU path: one mock at a time
    fp64 = None
    if args.fp64_mocks > 0:
        d64 = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F64, observer=obs)
        sc64 = pl.Scratch()
        plan64 = pl.bispec_plan(d64, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F64, sc64)
        order = np.argsort(sizes)
        pick = [int(order[len(order) // 2])] + [int(order[0])][: max(0, args.fp64_mocks - 1)]
        g, r = gpu_mocks[pick[0]]
        pl.measure_pk_bk(d64, g, r, bins, plan64, scratch=sc64)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        res64 = {}
        for k in pick:
            g, r = gpu_mocks[k]
            res64[k] = pl.measure_pk_bk(d64, g, r, bins, plan64, scratch=sc64)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t) / len(pick)
        fp64 = {"catalogs_per_s": 1.0 / per, "mocks_timed": [int(sizes[k]) for k in pick],
                "speedup_fp32_batched": value * per}
        kmin = int(np.argmin(sizes[: args.mocks]))
        if kmin in res64:
            e64 = smallest_mock_vs_oracle(mocks, sizes, {kmin: (res64[kmin]["pk"], res64[kmin]["bk"])},
                                          args.mocks)
            fp64["rel_error_vs_oracle"] = e64
        del sc64
    cpu = None if args.no_cpu else cpu_baseline(mocks, sizes, log=lambda *m: log(args, *m),
                                                workers=args.cpu_workers or None)
    copy_gbs = copy_rate_gbs()
    log(args, f"plain streaming copy: {copy_gbs:.0f} GB/s")

    # kernel times: the batch once more, eagerly on a single stream (kernels
    # unshared, so each launch's time is that kernel's own), every launch of the
    # timed classes bracketed by HIP events on its launch stream.  This is the
    # last GPU work of the run: the roofline kernel's launches are the last ones
    # of that kernel in a rocprofv3 trace of the same command.
    # (the same engine as the timed replays, on one stream)
    mask = sum(1 << v for v in L.KT.values())
    if native:
        single = pl.NativeBatch(desc, bins, plan, nstreams=1, max_ngal=max(int(g.shape[1]) for g, _ in gpu_mocks),
                                max_nran=max(int(r.shape[1]) for _, r in gpu_mocks))

        def single_run():
            single.run(gpu_mocks, outs)
    else:
        single = pl.Batch(1)

        def single_run():
            single.run(desc, gpu_mocks, bins, plan, outs)
    single_run()  # scratch of the single stream
    torch.cuda.synchronize()
    L.check(L.lib.cnpc_ktimer_start(mask, 1 << 16))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    single_run()
    e1.record()
    kern = ktimer_read(L)
    ms_instr = e0.elapsed_time(e1)
    stages = stage_roofline(model, kern)
    roof = paint_roofline(model, kern["paint"])
    roof["kernel"] = KERNEL_OF_CLASS["paint"]
    roof["launches"] = kern["paint"]["launches"]
    roof["traffic"] = measured_traffic(roof["kernel"])
    if roof["traffic"] is not None:
        roof["traffic_over_algorithmic"] = roof["traffic"] / roof["per_launch"]
    roof["copy_gbs"] = copy_gbs
    roof["frac_of_copy"] = roof["achieved"] / copy_gbs
    roof["durations_from"] = (f"HIP events around each launch of a single-stream eager pass of the "
                              f"batch run last ({ms_instr:.1f} ms for the batch)")
    kern_ms = {k: round(v["ms"], 3) for k, v in kern.items()}

    hbm_bytes = float(np.sum([pipeline_bytes(int(sz), 10 * int(sz)) for sz in sizes[: args.mocks]]))
    line = {
        "metric": "P_l/B_l catalogs/s at 256^3 (batched FP32)",
        "value": value,
        "unit": "catalogs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms_median": float(np.median(step_ms)),
        "timed_outputs_vs_eager": replay_err,
        "step_ms_min": float(np.min(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.PREC_F32 else "f32+bf16x3",
        "graph": "none" if args.no_graph else ("per-stream" if args.graph_per_stream else "one"),
        "engine": "cnpc_batch" if native else "python Batch",
        "streams": nstreams,
        "placement": args.balance,
        "tuning": tuning,
        "setup_s": {"upload": round(t_up, 3), "upload_gbs_pcie": round(up_bytes / t_up / 1e9, 2),
                    "bispec_plan": round(t_plan, 3), "first_eager_batch": round(t_eager, 3),
                    "graph_capture": None if t_cap is None else round(t_cap, 3)},
        "data": "synthetic lognormal mocks (seeded), resident in HBM",
        "config": {"workload": "64 uneven lognormal mocks (N_g 1e6-8e6 log-uniform, 10x randoms), "
                               "256^3 TSC + interlacing, L=1000, P_0,2,4 + Scoccimarro B_0 (20 bins, "
                               "dk=0.01) with analytic shot noise",
                   "global_batch": args.mocks, "nmesh": 256, "particles_total": ntot},
        "pipeline_hbm_frac": (hbm_bytes / (ms_step / 1e3)) / (HBM_PEAK_GBS * 1e9),
        "hbm_copy_gbs": copy_gbs,
        "pipeline_copy_frac": (hbm_bytes / (ms_step / 1e3)) / (copy_gbs * 1e9),
        "kernels_ms_per_step": kern_ms,
        "roofline": roof,
        "roofline_by_stage": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                                  for kk, vv in v.items()} for k, v in stages.items()},
        "rel_error_vs_oracle": vs_oracle,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def smallest_mock_vs_oracle(mocks, sizes, eager, nmocks):
    """Errors of the batch's outputs for its smallest mock against the stored
    FP64 oracle outputs of that catalog (tests/golden/oracle_c4min.json,
    written by the oracle alone), when the catalog digest matches."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "oracle_c4min.json")
    k = int(np.argmin(sizes[:nmocks]))
    if not os.path.exists(path) or k != int(np.argmin(sizes)):
        return None
    with open(path) as fh:
        fx = json.load(fh)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(mocks[k][0]).tobytes())
    h.update(np.ascontiguousarray(mocks[k][1]).tobytes())
    if h.hexdigest() != fx["catalog_sha256"]:
        return {"error": "catalog digest differs from the fixture's"}
    pk, bk = eager[k][0].cpu().numpy(), eager[k][1].cpu().numpy()
    raw, shot = np.asarray(fx["B0"]["raw"]), np.asarray(fx["B0"]["shot"])
    out = {f"P{l}": rel_err(pk[row], fx["pk"][f"P{l}"]) for row, l in enumerate((0, 2, 4))}
    out.update({"B0_raw": rel_err(bk[0], raw), "B0_shot": rel_err(bk[1], shot), "B0": rel_err(bk[2], raw - shot)})
    return {"mock_ng": int(sizes[k]), "errors": out}


def rel_err(a, b):
    """max |a - b| / max |b| over a multipole vector."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def single_config(args):
    """One catalog of configuration c1, c2, c3 or c5 (seeded lognormal galaxies
    and uniform randoms of the configuration's size): seconds per catalog of
    every precision form (catalogs resident in HBM, plans built beforehand) and
    the relative errors of FP32 and split-BF16 against the FP64 path."""
    import torch
    import paper_2605_04864_amd as cn
    from paper_2605_04864_amd import _lib as L
    from paper_2605_04864_amd import pipeline as pl
    import synthcat

    spec = synthcat.config_spec(args.config)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    g = synthcat.lognormal_catalog(spec.ngal, spec.boxsize, 1000 * args.config)
    r = synthcat.random_catalog(spec.nran, 1000 * args.config + 1)
    import hashlib
    hs = hashlib.sha256()
    hs.update(np.ascontiguousarray(g).tobytes())
    hs.update(np.ascontiguousarray(r).tobytes())
    g_sha = hs.hexdigest()
    log(args, f"generated c{args.config} catalogs in {time.time() - t0:.1f}s")
    gd, rd = torch.from_numpy(g).to(dev), torch.from_numpy(r).to(dev)
    del g, r
    obs = synthcat.observer_position()
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    descs = {dt: cn.mesh_desc(spec.nmesh, spec.boxsize, assign=spec.assign, interlace=spec.interlace,
                              dtype=dt, observer=obs) for dt in (L.F32, L.F64)}
    # (name, precision form, callable returning {output: tensor})
    jobs = []
    if args.config in (1, 2):
        modified = args.config == 2

        def pk(dt):
            def run():
                res = pl.measure_pk(descs[dt], gd, rd, bins, ells=spec.ells, modified=modified)
                keys = pl.PK_ROWS if modified else ("P0", "P2", "P4")
                return {k: res[k] for k in keys}
            return run
        jobs += [("pk", "f64", pk(L.F64)), ("pk", "f32", pk(L.F32))]
        # odd multipoles alongside the even ones, and the cross multipoles of
        # two tracers (alternate galaxies, each with alternate randoms)
        ga, gb = gd[:, 0::2].contiguous(), gd[:, 1::2].contiguous()
        ra, rb = rd[:, 0::2].contiguous(), rd[:, 1::2].contiguous()

        def pk_odd(dt):
            def run():
                res = pl.measure_pk(descs[dt], gd, rd, bins, ells=(0, 1, 2, 3, 4))
                return {k: res[k] for k in ("P0", "P1", "P2", "P3", "P4")}
            return run

        def pk_cross(dt):
            def run():
                res = pl.measure_pk_cross(descs[dt], (ga, ra), (gb, rb), bins, ells=(0, 1, 2, 3, 4))
                return {k: res[k] for k in ("P0", "P1", "P2", "P3", "P4")}
            return run
        jobs += [("pk_odd", "f64", pk_odd(L.F64)), ("pk_odd", "f32", pk_odd(L.F32)),
                 ("pk_cross", "f64", pk_cross(L.F64)), ("pk_cross", "f32", pk_cross(L.F32))]
    else:
        ests = ([("B0", L.EST_SCOCCIMARRO, 0), ("B2", L.EST_SCOCCIMARRO, 2), ("B202", L.EST_TRIPOSH, 2)]
                if args.config == 3 else [("B202", L.EST_TRIPOSH, 2)])
        forms = [("f64", L.F64, L.PREC_F64), ("f32", L.F32, L.PREC_F32), ("bf16x3", L.F32, L.PREC_BF16X3)]

        def bk(dt, prec, est, ell, noise="analytic"):
            def run():
                res = pl.measure_bk(descs[dt], gd, rd, bins, estimator=est, ell=ell, precision=prec,
                                    noise=noise)
                return {"raw": res["raw"], "shot": res["shot"], "value": res["value"]}
            return run
        for name, est, ell in ests:
            jobs += [(name, f, bk(dt, prec, est, ell)) for f, dt, prec in forms]
        # TripoSH with the FFT-method i = j != k noise term
        jobs += [("B202_fft_noise", f, bk(dt, prec, L.EST_TRIPOSH, 2, "fft")) for f, dt, prec in forms]
        if spec.nbins <= 22:
            # Sugiyama B_l1l2L over every pair of shells (split BF16 holds up to 22 shells)
            def sugi(dt, prec, l1, l2, Lm):
                def run():
                    res = pl.measure_sugiyama(descs[dt], gd, rd, bins, l1, l2, Lm, precision=prec)
                    return {"raw": res["raw"], "shot": res["shot"], "value": res["value"]}
                return run
            for l1, l2, Lm in ((0, 0, 0), (2, 0, 2), (2, 2, 0)):
                jobs += [(f"Sugiyama_B{l1}{l2}{Lm}", f, sugi(dt, prec, l1, l2, Lm)) for f, dt, prec in forms]

            def sugi_fft(dt, prec):
                def run():
                    res = pl.measure_sugiyama(descs[dt], gd, rd, bins, 2, 0, 2, precision=prec, noise="fft")
                    return {"raw": res["raw"], "shot": res["shot"], "value": res["value"]}
                return run
            jobs += [("Sugiyama_B202_fft_noise", f, sugi_fft(dt, prec)) for f, dt, prec in forms]
    times, outs = {}, {}
    for name, form, run in jobs:
        outs[(name, form)] = {k: v.detach().cpu().numpy() for k, v in run().items()}  # warm: plans, scratch
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        times.setdefault(name, {})[form] = e0.elapsed_time(e1) / 1e3 / args.reps
        log(args, f"c{args.config} {name} {form}: {times[name][form]:.4f} s per catalog")
    errors = {}
    for (name, form), o in outs.items():
        if form == "f64":
            continue
        ref = outs[(name, "f64")]
        errors.setdefault(name, {})[form] = {k: rel_err(o[k], ref[k]) for k in o}
    oracle_err = oracle_fixture_errors(args.config, g_sha, outs)
    line = {
        "metric": "seconds per catalog",
        "config": {"workload": spec.name, "ngal": spec.ngal, "nran": spec.nran, "nmesh": spec.nmesh,
                   "boxsize": spec.boxsize, "nbins": spec.nbins, "dk": spec.dk},
        "n_gpus": 1,
        "data": "synthetic lognormal galaxies + uniform randoms (seeded), resident in HBM",
        "reps": args.reps,
        "seconds_per_catalog": times,
        "rel_error_vs_fp64": errors,
        "rel_error_vs_oracle": oracle_err,
    }
    print(json.dumps(line))


def oracle_fixture_errors(config, sha, outs):
    """Errors of every form against the stored FP64 oracle outputs of this
    catalog (tests/golden/oracle_c2.json, oracle_c3.json, written by the
    oracle alone), when they exist and their catalog digest matches."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", f"oracle_c{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        fx = json.load(fh)
    if fx.get("catalog_sha256") != sha:
        return {"error": "catalog digest differs from the fixture's"}
    res = {}
    for (name, form), o in outs.items():
        if name == "pk" and "pk" in fx:
            res.setdefault(name, {})[form] = {k: rel_err(o[k], fx["pk"][k]) for k in o if k in fx["pk"]}
        key = {"B0": "B0", "B2": "B2", "B202": "BB202"}.get(name)
        if key and key in fx:
            raw, shot = np.asarray(fx[key]["raw"]), np.asarray(fx[key]["shot"])
            res.setdefault(name, {})[form] = {"raw": rel_err(o["raw"], raw), "shot": rel_err(o["shot"], shot),
                                              "value": rel_err(o["value"], raw - shot)}
    return res


def ktimer_read(L):
    """Stop the library's kernel timer: {class: {"ms": total, "launches": n}}."""
    ms_cls = (C.c_double * 16)()
    n_cls = (C.c_int64 * 16)()
    L.check(L.lib.cnpc_ktimer_stop(ms_cls, n_cls))
    return {k: {"ms": ms_cls[v], "launches": n_cls[v]} for k, v in L.KT.items()}


def stage_roofline(model, kern):
    """Achieved rate of every stage over the summed time of its kernel classes
    in one step: algorithmic bytes (contraction: MFMA flops) of the byte model
    over that time."""
    out = {}
    for st, cls in STAGE_CLASSES.items():
        ms = sum(kern[c]["ms"] for c in cls if c in kern)
        launches = sum(kern[c]["launches"] for c in cls if c in kern)
        if ms <= 0:
            continue
        if st == "intermediate":
            out[st] = {"classes": list(cls), "ms": ms, "launches": launches, "algorithmic": 0.0}
            continue
        if st == "contract":
            ach = model["contract_flops"] / (ms * 1e-3) / 1e12
            out[st] = {"bound": "mfma", "achieved": ach, "peak": PEAKS_TFLOPS["bf16"], "unit": "TFLOP/s",
                       "frac": ach / PEAKS_TFLOPS["bf16"], "ms": ms, "launches": launches}
            continue
        if st == "bin":
            # the byte model reads 16 full half-complex spectra; the design bins
            # band spectra (|n_i| < band), far fewer bytes: no rate is claimed
            out[st] = {"ms": ms, "launches": launches, "model_bytes": model[st],
                       "note": "band-pruned: reads less than the model's 16C"}
            continue
        ach = model[st] / (ms * 1e-3) / 1e9
        out[st] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": ach / HBM_PEAK_GBS, "ms": ms, "launches": launches, "classes": list(cls)}
    return out


def paint_roofline(model, kv):
    """The dominant kernel, the particle painter: one launch paints one catalog
    (both interlacing phases), algorithmic bytes 12 per particle of the launch
    plus its half of the mock's 4R mesh writes; per launch the step's paint
    bytes over its launches, over the average launch duration."""
    per_launch = model["paint"] / kv["launches"]
    avg_ms = kv["ms"] / kv["launches"]
    ach = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "avg_launch_ms": avg_ms, "per_launch": per_launch}


# kernel behind each timer class
KERNEL_OF_CLASS = {"paint": "k_paint_tiles_u32", "sort": "k_bucket_pass", "fold": "k_fold_zr2c",
                   "zr2c": "k_zpass_ylm_rr", "col": "k_colpass_rr", "zc2r": "k_zpass_c2r",
                   "contract": "k_contract_mfma", "bin": "k_bin", "sums": "k_catalog_sums"}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    `kernel` (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated), or None when
    there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{kernel}_traffic_256c_64mocks.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), vals.get("source", ""))
    if not os.path.exists(src):
        return None
    with open(src, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != vals.get("source_sha256"):
            return None
    return float(vals["bytes_per_launch"])


CPU_SLICE = 64  # the bounded sample paints and sums 1/64 of each picked mock


def cpu_picks(sizes):
    """The mocks the oracle is timed on: smallest, the two medians, largest."""
    order = np.argsort(sizes)
    m = len(order)
    return [int(order[0]), int(order[(m - 1) // 2]), int(order[m // 2]), int(order[-1])]


def oracle_sample(slices, n=256, box=1000.0):
    """One bounded, single-threaded sample of the FP64 oracle on the headline
    workload (P_0,2,4 by measure_pk and B_0 by measure_bk, as the oracle runs
    them: each sums and paints the catalogs itself; 12 single-catalog paintings
    of 6 (N_g + N_r) particles per mock in all).

    Per picked mock: the catalog sums of both calls and one painting of its
    random catalog, on a slice.  Once: the 9 de-interlacing FFTs, 14 Y_lm-
    weighted FFTs, 40 shell / indicator inverse FFTs, 2 x 825 triple sums and
    the binnings, one instance each, scaled by its repeat count."""
    import synthcat
    from oracle import bispectrum as obk
    from oracle import mesh as oms
    from oracle import spectra as osp
    from oracle.catalog import catalog_norms
    from oracle.ylm import Ylm
    obs = synthcat.observer_position()
    sums_s, paint_s, paint_n = [], [], []
    for g, r in slices:
        t = time.perf_counter()
        catalog_norms(g, None, r, None, box, obs, (0, 2, 4))
        catalog_norms(g, None, r, None, box, obs, (0,))
        sums_s.append(time.perf_counter() - t)
        t = time.perf_counter()
        oms.paint(r, None, n, oms.TSC, 0.5)
        paint_s.append(time.perf_counter() - t)
        paint_n.append(int(r.shape[1]))
    mesh = np.random.default_rng(0).normal(size=(n, n, n))
    parts = {}
    t = time.perf_counter()
    D = np.fft.fftn(mesh)
    parts["deinterlace_ffts"] = (time.perf_counter() - t) * 9
    rvec = osp.line_of_sight(n, box, obs)
    kvec = osp.kvectors(n, box)
    t = time.perf_counter()
    S = np.fft.fftn(mesh * Ylm(2, 1, rvec))
    np.conj(Ylm(2, 1, kvec)) * S
    parts["ylm_weighted_ffts"] = (time.perf_counter() - t) * 14
    del S, rvec, kvec
    bins = osp.Bins(0.0, 0.01, 20, box, n)
    t = time.perf_counter()
    X = obk.shell_field(D, bins.shell_index(), 10)
    parts["shell_and_indicator_iffts"] = (time.perf_counter() - t) * 40
    t = time.perf_counter()
    for _ in range(8):
        obk.triple_sum(X, X, X)
    parts["triple_sums"] = (time.perf_counter() - t) / 8 * 825 * 2
    t = time.perf_counter()
    bins.shell_mean(np.real(D * np.conj(D)))
    parts["binning"] = (time.perf_counter() - t) * 8
    return {"particles": [int(g.shape[1] + r.shape[1]) for g, r in slices], "sums_s": sums_s,
            "paint_particles": paint_n, "paint_s": paint_s, "mesh_parts_s": parts}


def fit_line(x, y):
    """Least-squares a, b of y = a x + b."""
    A = np.vstack([np.asarray(x, float), np.ones(len(x))]).T
    a, b = np.linalg.lstsq(A, np.asarray(y, float), rcond=None)[0]
    return float(a), float(b)


def sample_estimate(res, sizes):
    """Seconds per catalog of every mock from one oracle sample, as the line
    a (N_g + N_r) + b: a = 6 a_paint + a_sums, b = 12 b_paint + b_sums + the
    mesh stages (a_paint, b_paint: the painting's per-particle and per-call
    cost; a_sums, b_sums: the two catalog sums'), N_r = 10 N_g."""
    ap, bp = fit_line(res["paint_particles"], res["paint_s"])
    asum, bsum = fit_line(res["particles"], res["sums_s"])
    mesh_s = float(sum(res["mesh_parts_s"].values()))
    a = 6 * ap + asum
    b = 12 * bp + bsum + mesh_s
    per = [a * 11 * float(sz) + b for sz in sizes]
    return per, {"a_s_per_particle": a, "b_s": b, "paint_a_s": ap, "paint_b_s": bp, "sums_a_s": asum,
                 "mesh_s": mesh_s}


def _sample_worker(path):
    """Child process of the all-core sample: one oracle sample on the slices in
    `path` (an .npz the parent wrote), result as one JSON line."""
    z = np.load(path)
    slices = [(z[f"g{i}"], z[f"r{i}"]) for i in range(len([k for k in z.files if k.startswith("g")]))]
    print(json.dumps(oracle_sample(slices)))


def cpu_baseline(mocks, sizes, log=print, workers=None):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    Mocks: smallest, two medians, largest.  The particle stages run on 1/64 of
    each (the slope a of seconds = a (N_g + N_r) + b comes from these four
    sizes), the mesh stages once; the line gives every mock's seconds and the
    64-mock total.  Single-threaded (FFT and BLAS threads = 1), then the same
    sample in `workers` concurrent processes (all cores of the GPU's share of
    the host): the all-core throughput is workers / the mean per-process
    seconds per catalog."""
    import subprocess
    import tempfile
    picks = cpu_picks(sizes)
    slices = [(np.ascontiguousarray(mocks[k][0][:, : mocks[k][0].shape[1] // CPU_SLICE]),
               np.ascontiguousarray(mocks[k][1][:, : mocks[k][1].shape[1] // CPU_SLICE])) for k in picks]
    t = time.perf_counter()
    single = oracle_sample(slices)
    t_single = time.perf_counter() - t
    per, fit = sample_estimate(single, sizes)
    total = float(np.sum(per))
    log(f"cpu oracle, one thread: {total / len(sizes):.1f} s per mean catalog "
        f"({t_single:.1f} s sample); fit a={fit['a_s_per_particle']:.3e} s/particle, b={fit['b_s']:.1f} s")
    workers = workers or min(os.cpu_count() or 1, 16)
    allcore = None
    if workers > 1:
        with tempfile.TemporaryDirectory(dir="/tmp") as td:
            path = os.path.join(td, "slices.npz")
            np.savez(path, **{f"g{i}": g for i, (g, _) in enumerate(slices)},
                     **{f"r{i}": r for i, (_, r) in enumerate(slices)})
            env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
            cmd = [sys.executable, os.path.abspath(__file__), "--cpu-sample-worker", path]
            t = time.perf_counter()
            procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, env=env, text=True) for _ in range(workers)]
            outs = [p.communicate()[0] for p in procs]
            t_all = time.perf_counter() - t
            if all(p.returncode == 0 for p in procs):
                ests = [float(np.sum(sample_estimate(json.loads(o.strip().splitlines()[-1]), sizes)[0]))
                        for o in outs]
                mean_total = float(np.mean(ests))
                allcore = {"value": workers * len(sizes) / mean_total, "cores": workers,
                           "seconds_per_mean_catalog_per_process": mean_total / len(sizes),
                           "sample_wall_s": round(t_all, 1)}
                log(f"cpu oracle, {workers} processes: {allcore['value']:.4f} catalogs/s")
            else:
                log("cpu oracle all-core sample failed: " + str([p.returncode for p in procs]))
    one = {"value": len(sizes) / total, "cores": 1, "seconds_per_mean_catalog": total / len(sizes),
           "sample_wall_s": round(t_single, 1)}
    best = allcore or one
    return {"value": best["value"], "unit": "catalogs/s", "cores": best["cores"], "kind": "oracle",
            "sample": (f"oracle measure_pk (P_0,2,4) + measure_bk (B_0) as they stand, 256^3 TSC + interlacing; "
                       f"mocks {[int(sizes[k]) for k in picks]} (N_g: smallest, two medians, largest of the "
                       f"{len(sizes)}); catalog sums and one painting timed on 1/{CPU_SLICE} of each (their "
                       f"per-particle and per-call costs fitted over the four sizes), FFT / shell / triple-sum / "
                       f"binning stages timed once each and scaled by their repeat counts; seconds per mock "
                       f"a (N_g + N_r) + b, summed over all {len(sizes)} mocks; on the build host this sample "
                       f"estimates 22% less time than the oracle takes on whole mocks "
                       f"(profiles/cpu_oracle_whole_mocks_c4.txt)"),
            "single_thread": one, "all_cores": allcore, "fit": fit,
            "parts_s": {k: round(v, 2) for k, v in single["mesh_parts_s"].items()},
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def cpu_whole(args):
    """The oracle on whole mocks (smallest, two medians, largest), one thread,
    against the bounded sample's estimate for the same mocks on the same host."""
    import synthcat
    from oracle.pipeline import MeshConfig, measure_bk, measure_pk
    from oracle import mesh as oms
    sizes = synthcat.mock_sizes_c4(64)
    picks = cpu_picks(sizes)
    cfg = MeshConfig(1000.0, 256, oms.TSC, True, synthcat.observer_position())
    whole = []
    slices = []
    for k in picks:
        ng = int(sizes[k])
        g = synthcat.lognormal_catalog(ng, 1000.0, 4000 + 2 * k)
        r = synthcat.random_catalog(10 * ng, 4000 + 2 * k + 1)
        slices.append((np.ascontiguousarray(g[:, : ng // CPU_SLICE]),
                       np.ascontiguousarray(r[:, : r.shape[1] // CPU_SLICE])))
        t = time.perf_counter()
        measure_pk(g, None, r, None, cfg, 0.0, 0.01, 20, ells=(0, 2, 4))
        measure_bk(g, None, r, None, cfg, 0.01, 20, ells=(0,), scoccimarro=(0,), triposh=())
        whole.append(time.perf_counter() - t)
        log(args, f"whole mock N_g={ng}: {whole[-1]:.1f} s")
        del g, r
    npart = [11 * int(sizes[k]) for k in picks]
    a, b = fit_line(npart, whole)
    est, fit = sample_estimate(oracle_sample(slices), sizes)
    print(json.dumps({"kind": "oracle whole mocks, one thread", "mocks_ng": [int(sizes[k]) for k in picks],
                      "seconds": [round(x, 1) for x in whole], "fit_a_s_per_particle": a, "fit_b_s": b,
                      "total_64_mocks_s": float(a * 11 * np.sum(sizes) + 64 * b),
                      "catalogs_per_s": 64 / float(a * 11 * np.sum(sizes) + 64 * b),
                      "sample_estimate_same_mocks_s": [round(est[k], 1) for k in picks],
                      "sample_total_64_mocks_s": float(np.sum(est)), "sample_fit": fit,
                      "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}))


def _cpu_model():
    """The lscpu model name (else /proc/cpuinfo's)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
