"""Parity under every value of the library's tuning knobs, and the autotuner.

Each knob only changes launch shapes, so every setting must meet the same bar
against the FP64 oracle as the defaults: the FFT, Y_lm and power-spectrum
cases rerun with the LDS Stockham passes and other column tile widths, the
bucketed sort with other particles per thread and workgroup sizes (paint
stays bit-exact), and the
split-BF16 contraction with every point-group split on 20 shells (210 shell
pairs: 7 pair tiles, so 2, 4 or 7 tiles per wave; 20 or 40 fields).
"""

import contextlib

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import autotune  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
from oracle.pipeline import MeshConfig, measure_bk  # noqa: E402
import test_gpu_parity as P  # noqa: E402


@contextlib.contextmanager
def knobs(**kv):
    autotune.set_knobs(kv)
    try:
        yield
    finally:
        autotune.reset_knobs()


@pytest.mark.parametrize("n", [64, 128, 256])
def test_fft_full_stockham_only(n):
    with knobs(fft_passes=1):
        P.test_fft_full_r2c_c2r(n, L.F32)


@pytest.mark.parametrize("setting", [{"fft_passes": 1}, {"fft_passes": 1, "fft_col_w": 4},
                                     {"fft_col_w": 1}, {"fft_col_w": 64}])
@pytest.mark.parametrize("n,band", [(64, 16), (128, 32), (256, 32)])
def test_fft_band_knobs(n, band, setting):
    with knobs(**setting):
        P.test_fft_band_r2c_c2r(n, band, L.F32)


@pytest.mark.parametrize("n,band,dtype", [(64, 16, L.F64), (256, 32, L.F32)])
def test_ylm_band_stockham_only(n, band, dtype):
    with knobs(fft_passes=1):
        P.test_ylm_r2c_band(n, band, dtype, (2, 4), None)


@pytest.mark.parametrize("n,band,ells,los", [(256, 32, (2, 4), None), (64, 16, (1, 2, 3, 4), None),
                                             (256, 32, (2, 4), P.YLM_LOS)])
def test_ylm_band_per_field(n, band, ells, los):
    """CNPC_TUNE_YLM_BASIS 1: one z transform per field in place of the
    z-power bases."""
    with knobs(ylm_basis=1):
        P.test_ylm_r2c_band(n, band, L.F32, ells, los)


def test_measure_pk_ylm_per_field():
    with knobs(ylm_basis=1):
        P.test_measure_pk_vs_oracle(64, L.TSC, True, L.F32)


def test_measure_pk_stockham_only():
    """n = 64 with interlacing: the deinterlace takes its plain 3-D transform
    route instead of the fused x pass."""
    with knobs(fft_passes=1):
        P.test_measure_pk_vs_oracle(64, L.TSC, True, L.F32)


@pytest.mark.parametrize("threads", [512, 1024])
@pytest.mark.parametrize("per", [1, 2, 4])
@pytest.mark.parametrize("case", ["dense128", "sparse256_weighted", "one_tile256"])
def test_paint_sort_per(case, per, threads):
    with knobs(sort_per=per, sort_threads=threads):
        P.test_paint_bucketed_sort(case)


_ORACLE = {}


@pytest.mark.parametrize("kg", [0, 1, 2, 4])
@pytest.mark.parametrize("est,ell", [(L.EST_SCOCCIMARRO, 0), (L.EST_SCOCCIMARRO, 2)])
def test_contract_point_groups_20_shells(est, ell, kg):
    n, box = 64, 1000.0
    nb, dk = 20, 0.007
    g, r = P._cat(31, 30_000, 150_000)
    bins = cn.kbins(0.0, dk, nb)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=P.OBS)
    with knobs(contract_kg=kg):
        res = pl.measure_bk(d, P.dev(g), P.dev(r), bins, estimator=est, ell=ell, precision=L.PREC_BF16X3)
        raw, val = P.host(res["raw"]), P.host(res["value"])
    if (est, ell) not in _ORACLE:
        cfg = MeshConfig(box, n, L.TSC, True, P.OBS)
        sc = (ell,) if est == L.EST_SCOCCIMARRO else ()
        tr = (ell,) if est == L.EST_TRIPOSH else ()
        _ORACLE[(est, ell)] = measure_bk(g, None, r, None, cfg, dk, nb, ells=tuple(sorted({0, ell})),
                                         scoccimarro=sc, triposh=tr)
    ora = _ORACLE[(est, ell)]
    key = f"B{ell}" if est == L.EST_SCOCCIMARRO else f"BB{ell}0{ell}"
    assert P.rel(raw, ora[f"{key}_raw"]) < 1e-3
    assert P.rel(val, ora[key]) < 1e-3


@pytest.mark.parametrize("engine", ["torch", "native"])
def test_autotune_batch(tmp_path, engine):
    """The tuner returns a valid setting, leaves the knobs set to it, caches
    it, and the tuned batch gives the default batch's results."""
    n, box = 32, 1000.0
    bins = cn.kbins(0.0, 0.012, 4)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=P.OBS)
    cats = [P._cat(41 + 2 * k, 10_000 * (k + 1), 60_000 * (k + 1)) for k in range(3)]
    cats = [(P.dev(g), P.dev(r)) for g, r in cats]
    sc = pl.Scratch()
    plan = pl.bispec_plan(d, bins, L.EST_SCOCCIMARRO, 0, L.PREC_BF16X3, sc)
    ref = [pl.measure_pk_bk(d, g, r, bins, plan, scratch=sc) for g, r in cats]
    ref = [(P.host(o["pk"]).copy(), P.host(o["bk"]).copy()) for o in ref]
    path = str(tmp_path / "tune.json")
    try:
        res = autotune.tune_batch(d, cats, bins, plan, streams=(1, 2), reps=1, cache=path, engine=engine)
        assert res.streams in (1, 2) and not res.cached and len(res.trials) >= 5
        assert res.ms > 0 and res.default_ms > 0
        assert autotune.get_knobs() == res.knobs
        for k, v in res.knobs.items():
            assert v in L.TUNE[k][1]
        again = autotune.tune_batch(d, cats, bins, plan, streams=(1, 2), reps=1, cache=path, engine=engine)
        assert again.cached and again.knobs == res.knobs and again.streams == res.streams
        outs = [{"pk": torch.empty((9, 4), dtype=torch.float64, device="cuda"),
                 "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device="cuda")} for _ in cats]
        if engine == "native":
            pl.NativeBatch(d, bins, plan, nstreams=res.streams, max_ngal=max(g.shape[1] for g, _ in cats),
                           max_nran=max(r.shape[1] for _, r in cats)).run(cats, outs)
        else:
            pl.Batch(res.streams).run(d, cats, bins, plan, outs)
        torch.cuda.synchronize()
        for (pk, bk), o in zip(ref, outs):
            assert P.rel(P.host(o["pk"]), pk) < 1e-5
            assert P.rel(P.host(o["bk"]), bk) < 1e-3
    finally:
        autotune.reset_knobs()


@pytest.mark.parametrize("est,ell", [(L.EST_SCOCCIMARRO, 0), (L.EST_TRIPOSH, 2)])
def test_shell_c2r_inside_contraction(est, ell):
    """CNPC_TUNE_SHELL_FUSED: the split-BF16 contraction on the 128^3 grid of a
    256^3 mesh that runs the shells' c2r z pass itself gives the results of
    the real shell fields written first (same transforms, same contraction)."""
    n, box = 256, 1000.0
    bins = cn.kbins(0.0, 0.01, 20)
    g, r = P._cat(41, 200_000, 800_000)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=P.OBS)
    res = {}
    for v in (0, 1):
        with knobs(shell_fused=v):
            o = pl.measure_bk(d, P.dev(g), P.dev(r), bins, estimator=est, ell=ell, precision=L.PREC_BF16X3)
            res[v] = {k: P.host(o[k]) for k in ("raw", "shot", "value")}
    for k in ("raw", "shot", "value"):
        assert P.rel(res[0][k], res[1][k]) < 1e-12, k
