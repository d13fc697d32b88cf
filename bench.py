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
    ap.add_argument("--staged", action="store_true",
                    help="painting and spectra on separate streams (with --no-tune)")
    ap.add_argument("--balance", choices=["rr", "lpt", "mixed"], default="rr",
                    help="placement of the catalogs on the streams (see pipeline.Batch.assignment)")
    ap.add_argument("--tune-mocks", type=int, default=16, help="mocks per autotuner trial batch")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--fp64-mocks", type=int, default=2, help="mocks timed on the plain FP64 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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


def class_model(ng, nr, n=256, es=4, band=32, grid=128, nb=20, nfields=14, nphase=2):
    """Algorithmic HBM bytes (or MFMA flops) of one mock per kernel class of the
    path: every array read or written once by the kernels of that class."""
    ntiles, bvol = (n // 16) ** 3, 19 ** 3
    npart = ng + nr
    blocks = ntiles * nphase * bvol * es            # one catalog's tile blocks
    mesh = n ** 3 * es                               # one real mesh
    half = n * n * (n // 2) * 2 * es                 # one half-layout spectrum
    zb = n * n * band * 2 * es                       # one z-pruned band plane stack
    yb = n * 2 * band * band * 2 * es                # after the y pass
    xb = 4 * band ** 3 * 2 * es                      # band spectrum
    g3 = grid ** 3 * es
    gz = grid * grid * band * 2 * es
    gy = grid * 2 * band * band * 2 * es
    npairs = nb * (nb + 1) // 2
    return {
        "sums": 12 * npart,
        "sort": 2 * 24 * npart,
        "paint": 12 * npart + 2 * blocks,
        "fold": 2 * blocks + 2 * nphase * mesh,
        "zr2c": nphase * (mesh + half) + nphase * (mesh + zb) + (mesh + nfields * zb),
        "col": (nphase * 4 * half + nphase * (zb + 2 * yb + xb) + nfields * (zb + 2 * yb + xb)
                + 4 * half + nb * (xb + 2 * gy + gz)),
        "zc2r": (half + mesh) + nb * (gz + g3),
        "bin": (nfields + 4) * xb,
        "contract": 3 * 2.0 * npairs * nb * grid ** 3,   # MFMA flops (split bf16: 3 products)
    }


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


def main():
    args = parse()
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
    gpu_mocks = [(torch.from_numpy(g).to(dev), torch.from_numpy(r).to(dev)) for g, r in mocks]
    torch.cuda.synchronize()
    log(args, f"uploaded in {time.time() - t0:.1f}s")
    obs = synthcat.observer_position()
    bins = cn.kbins(0.0, 0.01, 20)
    prec = L.PREC_BF16X3 if args.precision == "bf16x3" else L.PREC_F32
    desc = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=obs)
    sc = pl.Scratch()
    plan = pl.bispec_plan(desc, bins, L.EST_SCOCCIMARRO, 0, prec, sc)
    outs = [{"pk": torch.empty((9, 20), dtype=torch.float64, device=dev),
             "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device=dev)} for _ in gpu_mocks]
    tuning = None
    nstreams = args.streams or 4
    staged = args.staged
    if not args.no_tune:
        from paper_2605_04864_amd import autotune
        tcat = gpu_mocks[: max(1, min(args.tune_mocks, len(gpu_mocks)))]
        res = autotune.tune_batch(desc, tcat, bins, plan, use_cache=False, reps=5,
                                  streams=(args.streams,) if args.streams else (1, 2, 3, 4, 6),
                                  log=lambda m: log(args, m), engine=args.engine)
        nstreams = res.streams
        staged = res.staged
        tuning = res.as_dict()
        tuning["batch_mocks"] = len(tcat)
        log(args, f"autotuned in {res.seconds:.1f}s: streams {res.streams}, staged {res.staged}, knobs {res.knobs}, "
                  f"{res.default_ms:.2f} -> {res.ms:.2f} ms per {len(tcat)} mocks")
    native = args.engine == "native" and not staged and not args.graph_per_stream and args.balance == "rr"
    if native:
        batch = pl.NativeBatch(desc, bins, plan, nstreams=nstreams,
                               max_ngal=max(int(g.shape[1]) for g, _ in gpu_mocks),
                               max_nran=max(int(r.shape[1]) for _, r in gpu_mocks))

        def step():
            batch.run(gpu_mocks, outs)
    else:
        batch = pl.Batch(nstreams, staged=staged, balance=args.balance)

        def step():
            batch.run(desc, gpu_mocks, bins, plan, outs)

    step()  # eager pass: plans, twiddles and scratch reach their final size
    torch.cuda.synchronize()
    eager = [(o["pk"].clone(), o["bk"].clone()) for o in outs]

    ntot = int(np.sum(sizes[: args.mocks]) * 11)
    models = [class_model(int(sz), 10 * int(sz), band=plan.band, grid=plan.grid)
              for sz in sizes[: args.mocks]]
    model = {k: float(np.sum([m[k] for m in models])) for k in models[0]}  # per step

    run = step
    if args.graph_per_stream and not args.no_graph and not staged:
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
        batch.capture(gpu_mocks, outs)
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
        for k in pick:
            g, r = gpu_mocks[k]
            pl.measure_pk_bk(d64, g, r, bins, plan64, scratch=sc64)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t) / len(pick)
        fp64 = {"catalogs_per_s": 1.0 / per, "mocks_timed": [int(sizes[k]) for k in pick],
                "speedup_fp32_batched": value * per}
        del sc64
    cpu = None if args.no_cpu else cpu_baseline(mocks, sizes, log=lambda *m: log(args, *m))

    # kernel times: the batch once more, eagerly on a single stream (kernels
    # unshared, so each launch's time is that kernel's own), every launch of the
    # timed classes bracketed by HIP events on its launch stream.  This is the
    # last GPU work of the run: the roofline kernel's launches are the last ones
    # of that kernel in a rocprofv3 trace of the same command.
    mask = sum(1 << v for v in L.KT.values())
    single = pl.Batch(1)
    single.run(desc, gpu_mocks, bins, plan, outs)  # scratch of the single stream
    torch.cuda.synchronize()
    L.check(L.lib.cnpc_ktimer_start(mask, 1 << 16))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    single.run(desc, gpu_mocks, bins, plan, outs)
    e1.record()
    kern = ktimer_read(L)
    ms_instr = e0.elapsed_time(e1)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    classes = {name: class_roofline(name, kv, model) for name, kv in kern.items()
               if kv["launches"] > 0 and kv["ms"] > 0}
    roof = dict(classes[dom])
    roof["kernel"] = KERNEL_OF_CLASS.get(dom, dom)
    roof["launches"] = kern[dom]["launches"]
    roof["traffic"] = measured_traffic(roof["kernel"])
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
        "staged": staged,
        "placement": args.balance,
        "tuning": tuning,
        "data": "synthetic lognormal mocks (seeded), resident in HBM",
        "config": {"workload": "64 uneven lognormal mocks (N_g 1e6-8e6 log-uniform, 10x randoms), "
                               "256^3 TSC + interlacing, L=1000, P_0,2,4 + Scoccimarro B_0 (20 bins, "
                               "dk=0.01) with analytic shot noise",
                   "global_batch": args.mocks, "nmesh": 256, "particles_total": ntot},
        "pipeline_hbm_frac": (hbm_bytes / (ms_step / 1e3)) / (HBM_PEAK_GBS * 1e9),
        "kernels_ms_per_step": kern_ms,
        "roofline": roof,
        "roofline_by_class": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                                  for kk, vv in v.items()} for k, v in classes.items()},
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


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
    line = {
        "metric": "seconds per catalog",
        "config": {"workload": spec.name, "ngal": spec.ngal, "nran": spec.nran, "nmesh": spec.nmesh,
                   "boxsize": spec.boxsize, "nbins": spec.nbins, "dk": spec.dk},
        "n_gpus": 1,
        "data": "synthetic lognormal galaxies + uniform randoms (seeded), resident in HBM",
        "reps": args.reps,
        "seconds_per_catalog": times,
        "rel_error_vs_fp64": errors,
    }
    print(json.dumps(line))


def ktimer_read(L):
    """Stop the library's kernel timer: {class: {"ms": total, "launches": n}}."""
    ms_cls = (C.c_double * 16)()
    n_cls = (C.c_int64 * 16)()
    L.check(L.lib.cnpc_ktimer_stop(ms_cls, n_cls))
    return {k: {"ms": ms_cls[v], "launches": n_cls[v]} for k, v in L.KT.items()}


def class_roofline(name, kv, model):
    """Achieved rate of one kernel class: algorithmic bytes (or MFMA flops) per
    launch from the per-step model over the average launch duration."""
    per_launch = model[name] / kv["launches"]
    avg_ms = kv["ms"] / kv["launches"]
    if name == "contract":
        ach = per_launch / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": PEAKS_TFLOPS["bf16"], "unit": "TFLOP/s",
                "frac": ach / PEAKS_TFLOPS["bf16"], "avg_launch_ms": avg_ms, "per_launch": per_launch}
    ach = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": avg_ms, "per_launch": per_launch}


# kernel behind each timer class (the dominant one is named in the roofline)
KERNEL_OF_CLASS = {"paint": "k_paint_tiles_u32", "sort": "k_partition", "fold": "k_fold_tiles",
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


def cpu_baseline(mocks, sizes, log=print):
    """FP64 oracle on a bounded sample of the smallest mock, extrapolated to the mean mock.

    Each oracle step is timed on a slice and scaled by the number of times the
    whole computation repeats it; the sum estimates seconds per catalog."""
    import synthcat
    from oracle import bispectrum as obk
    from oracle import mesh as oms
    from oracle import spectra as osp
    from oracle.catalog import catalog_norms
    from oracle.ylm import Ylm
    k = int(np.argmin(sizes))
    g, r = mocks[k]
    ng, nr = g.shape[1], r.shape[1]
    n, box = 256, 1000.0
    obs = synthcat.observer_position()
    parts = {}
    frac = 50
    t = time.perf_counter()
    catalog_norms(g[:, : ng // frac], None, r[:, : nr // frac], None, box, obs, (0, 2, 4))
    parts["catalog_sums"] = (time.perf_counter() - t) * frac
    t = time.perf_counter()
    oms.paint(r[:, : nr // 20], None, n, oms.TSC, 0.0)
    # 8 paintings (2 catalogs x 2 interlacing phases x {w, w^2}) of all particles
    parts["paint"] = (time.perf_counter() - t) * 20 * 8 * (ng + nr) / nr
    mesh = np.random.default_rng(0).normal(size=(n, n, n))
    t = time.perf_counter()
    D = np.fft.fftn(mesh)
    one_fft = time.perf_counter() - t
    parts["deinterlace_ffts"] = one_fft * 6  # (A, B, inverse) for delta and N
    rvec = osp.line_of_sight(n, box, obs)
    kvec = osp.kvectors(n, box)
    t = time.perf_counter()
    S = np.fft.fftn(mesh * Ylm(2, 1, rvec))
    acc = np.conj(Ylm(2, 1, kvec)) * S
    one_m = time.perf_counter() - t
    parts["ylm_weighted_ffts"] = one_m * 14  # 5 (l=2) + 9 (l=4) m values
    del S, acc, rvec, kvec
    bins = osp.Bins(0.0, 0.01, 20, box, n)
    t = time.perf_counter()
    shells = bins.shell_index()
    X = obk.shell_field(D, shells, 10)
    one_shell = time.perf_counter() - t
    parts["shell_and_indicator_iffts"] = one_shell * 40
    t = time.perf_counter()
    for _ in range(8):
        obk.triple_sum(X, X, X)
    parts["triple_sums"] = (time.perf_counter() - t) / 8 * 825 * 2  # signal + triangle counts
    t = time.perf_counter()
    bins.shell_mean(np.real(D * np.conj(D)))
    parts["binning"] = (time.perf_counter() - t) * 6
    # particle-proportional steps scaled from the sampled mock to the mean mock
    scale = float(np.mean(sizes)) / float(sizes[k])
    parts["catalog_sums"] *= scale
    parts["paint"] *= scale
    total = sum(parts.values())
    threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    log(f"cpu oracle estimate {total:.1f}s per catalog: " +
        ", ".join(f"{k}={v:.1f}" for k, v in parts.items()))
    return {"value": 1.0 / total, "unit": "catalogs/s", "cores": 1, "kind": "oracle",
            "sample": f"smallest mock (N_g={ng}, N_r={nr}), 256^3: each oracle step timed on a "
                      f"slice (1/50 of the catalog sums, 1/20 of one painting, one 256^3 FFT, one "
                      f"Y_lm-weighted FFT, one shell inverse FFT, 8 triple sums) and scaled by its "
                      f"repeat count; sums and painting then scaled to the mean mock "
                      f"(N_g={float(np.mean(sizes)):.3g}); numpy FFT single-threaded",
            "seconds_per_catalog": total, "parts_s": {k: round(v, 2) for k, v in parts.items()},
            "omp_threads_env": threads, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def _cpu_model():
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
