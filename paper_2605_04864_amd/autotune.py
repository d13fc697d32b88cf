"""Autotuner of the launch shapes of a batched measurement.

A candidate setting is timed the way a batch is meant to run: the catalogs of
the batch are measured once eagerly (plans, twiddles and scratch reach their
size), the batch is captured into one HIP graph, and the graph is replayed.
The setting is

  streams      streams a ``pipeline.Batch`` spreads the catalogs over
  fft_passes   register FFT passes (0) or LDS Stockham passes only (1)
  fft_col_w    columns per workgroup of the LDS column passes (0: library's)
  contract_kg  point groups per split-BF16 contraction workgroup (0: library's)
  sort_per     particles per thread of the sort scatter (0: library's)
  sort_threads threads per sort-scatter workgroup (0: library's)
  sort_fused   how the catalog sums and the first sort step share reads (0, 1, 2)
  fold_fused   fold inside the de-interlacing z passes (0) or meshes written (1)
  bucket       shape of the first sort step (0, 1, 2)

All but the stream count are the library's tuning knobs (``cnpc_tune_set``); the search
is one coordinate-descent sweep in that order, each value timed with the
others held at the best found so far, and a value replaces the incumbent only
when it is faster by more than ``min_gain``.  Every setting gives results
within the tolerance of the kernels involved (paint and binning counts are
identical), so tuning never changes what is measured, only how fast.  The
choice is cached per device and workload in a JSON file.
"""

from __future__ import annotations

import json
import os
import statistics
import time
from dataclasses import asdict, dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import _lib as L

KNOB_ORDER = ("fft_passes", "fft_col_w", "contract_kg", "sort_per", "sort_threads", "sort_fused", "fold_fused",
              "bucket", "ylm_basis", "shell_fused")
DEFAULT_STREAMS = 4


def get_knobs() -> Dict[str, int]:
    return {k: int(L.lib.cnpc_tune_get(L.TUNE[k][0])) for k in KNOB_ORDER}


def set_knobs(knobs: Dict[str, int]) -> None:
    for k, v in knobs.items():
        if k not in L.TUNE:
            raise KeyError(f"unknown tuning knob {k!r}")
        L.check(L.lib.cnpc_tune_set(L.TUNE[k][0], int(v)))


def reset_knobs() -> None:
    set_knobs({k: 0 for k in KNOB_ORDER})


def coordinate_descent(space: Dict[str, Sequence], start: Dict, measure: Callable[[Dict], float],
                       min_gain: float = 0.01) -> Tuple[Dict, float, List[Tuple[Dict, float]]]:
    """One sweep over the keys of `space` in order.  `measure(setting)` returns a
    cost (lower is better).  Returns (best setting, its cost, all trials)."""
    best = dict(start)
    best_t = measure(best)
    trials = [(dict(best), best_t)]
    for key, values in space.items():
        for v in values:
            if v == best.get(key):
                continue
            cand = dict(best)
            cand[key] = v
            t = measure(cand)
            trials.append((dict(cand), t))
            if t < best_t * (1.0 - min_gain):
                best, best_t = cand, t
    return best, best_t, trials


def signature(desc, plan, ncat: int, ells: Sequence[int]) -> str:
    """Cache key: device, library, mesh, band/grid of the plan and batch size."""
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return "|".join(str(x) for x in (
        dev, L.lib.cnpc_version().decode(), desc.n, desc.dtype, desc.assign, desc.interlace,
        plan.band, plan.grid, plan.nconf, plan.ell, plan.estimator, plan.precision, ncat,
        ",".join(map(str, ells))))


def _cache_path(path: Optional[str]) -> str:
    if path:
        return path
    env = os.environ.get("CNPC_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "cnpc", "autotune.json")


def _cache_load(path: str) -> Dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) and d.get("version") == 1 else {"version": 1, "entries": {}}
    except (OSError, ValueError):
        return {"version": 1, "entries": {}}


def _cache_store(path: str, sig: str, entry: Dict) -> None:
    d = _cache_load(path)
    d.setdefault("entries", {})[sig] = entry
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


@dataclass
class TuneResult:
    streams: int
    knobs: Dict[str, int]
    ms: float                  # per batch, best setting
    default_ms: float          # per batch, library defaults (DEFAULT_STREAMS if offered)
    seconds: float             # wall time of the search (0 when cached)
    cached: bool
    trials: List[Dict] = field(default_factory=list)

    def as_dict(self):
        d = asdict(self)
        d["trials"] = len(self.trials)
        return d


def time_batch(desc, catalogs, bins, plan, ells=(0, 2, 4), nstreams: int = DEFAULT_STREAMS,
               reps: int = 3, engine: str = "torch") -> float:
    """Median ms per graph replay of the whole batch under the current knobs
    (engine "native": the library's cnpc_batch graph; "torch": pipeline.Batch
    captured with torch.cuda.CUDAGraph)."""
    import torch
    from . import pipeline as pl
    dev = catalogs[0][0].device
    outs = [{"pk": torch.empty((9, bins.nbins), dtype=torch.float64, device=dev),
             "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device=dev)} for _ in catalogs]
    if engine == "native":
        batch = pl.NativeBatch(desc, bins, plan, ells=ells, nstreams=nstreams,
                               max_ngal=max(int(g.shape[1]) for g, _ in catalogs),
                               max_nran=max(int(r.shape[1]) for _, r in catalogs), device=dev)
        batch.run(catalogs, outs)
        torch.cuda.synchronize()
        batch.capture(catalogs, outs)
        replay = batch.replay
    else:
        batch = pl.Batch(nstreams, device=dev)
        batch.run(desc, catalogs, bins, plan, outs, ells)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            batch.run(desc, catalogs, bins, plan, outs, ells)
        replay = graph.replay
    replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, reps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        replay()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del replay, batch, outs
    return statistics.median(times)


def tune_batch(desc, catalogs, bins, plan, ells=(0, 2, 4), streams: Sequence[int] = (1, 2, 3, 4, 6),
               reps: int = 3, min_gain: float = 0.02, cache: Optional[str] = None,
               use_cache: bool = True, log: Optional[Callable[[str], None]] = None,
               engine: str = "torch") -> TuneResult:
    """Pick the stream count and knob values for batches like `catalogs` and
    leave the knobs set to the choice."""
    path = _cache_path(cache)
    sig = signature(desc, plan, len(catalogs), ells) + "|" + engine
    if use_cache:
        hit = _cache_load(path).get("entries", {}).get(sig)
        if hit:
            set_knobs(hit["knobs"])
            return TuneResult(int(hit["streams"]), dict(hit["knobs"]), float(hit["ms"]), float(hit["default_ms"]),
                              0.0, True, [])
    space = {"streams": list(streams)}
    for k in KNOB_ORDER:
        space[k] = list(L.TUNE[k][1]) if k != "fft_col_w" else [0, 4, 8, 16, 32]
    s0 = DEFAULT_STREAMS if DEFAULT_STREAMS in streams else streams[0]
    start = {"streams": s0, **{k: 0 for k in KNOB_ORDER}}

    def measure(s):
        set_knobs({k: s[k] for k in KNOB_ORDER})
        t = time_batch(desc, catalogs, bins, plan, ells, s["streams"], reps, engine=engine)
        if log:
            log(f"autotune {s} -> {t:.3f} ms")
        return t

    t0 = time.time()
    try:
        best, best_t, trials = coordinate_descent(space, start, measure, min_gain)
    except BaseException:
        reset_knobs()
        raise
    knobs = {k: int(best[k]) for k in KNOB_ORDER}
    set_knobs(knobs)
    res = TuneResult(int(best["streams"]), knobs, float(best_t), float(trials[0][1]), time.time() - t0, False,
                     [dict(s, ms=t) for s, t in trials])
    if use_cache:
        _cache_store(path, sig, {"streams": res.streams, "knobs": knobs, "ms": res.ms,
                                 "default_ms": res.default_ms})
    return res
