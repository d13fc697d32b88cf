"""Sugiyama bispectrum multipoles B_l1l2L against the FP64 oracle, through the
C ABI: raw estimator, analytic shot noise and their difference for every
pair of shells, and the same with the FFT-method i = j != k noise term, in
FP64 (1e-10), FP32 (1e-5) and split BF16 (1e-3), relative to the largest
magnitude; B_000 also against the compressed TripoSH BB_000 of the library
(the same estimator), with both noise methods."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
from oracle.pipeline import MeshConfig, measure_sugiyama  # noqa: E402
import test_gpu_parity as P  # noqa: E402

_ORA = {}
FORMS = {"f64": (L.F64, L.PREC_F64, 1e-10), "f32": (L.F32, L.PREC_F32, 1e-5), "bf16": (L.F32, L.PREC_BF16X3, 1e-3)}


def _oracle(l1, l2, Lm, n=32, nb=4, dk=0.012, seed=9):
    key = (l1, l2, Lm, n, nb, dk, seed)
    if key not in _ORA:
        g, r = P._cat(seed, 30_000, 150_000)
        cfg = MeshConfig(1000.0, n, L.TSC, True, P.OBS)
        _ORA[key] = (g, r, measure_sugiyama(g, None, r, None, cfg, dk, nb, l1, l2, Lm, fft_noise=True))
    return _ORA[key]


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("l1,l2,Lm", [(0, 0, 0), (2, 0, 2), (2, 2, 0), (2, 2, 2), (1, 1, 2)])
def test_sugiyama_fft_noise_vs_oracle(l1, l2, Lm, form):
    n, nb, dk = 32, 4, 0.012
    g, r, ora = _oracle(l1, l2, Lm)
    dt, prec, tol = FORMS[form]
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dt, observer=P.OBS)
    bins = cn.kbins(0.0, dk, nb)
    res = pl.measure_sugiyama(d, P.dev(g), P.dev(r), bins, l1, l2, Lm, precision=prec, noise="fft")
    assert P.rel(P.host(res["raw"]), ora["raw"]) < tol
    assert P.rel(P.host(res["shot"]), ora["shot_fft"]) < tol
    assert P.rel(P.host(res["value"]), ora["value_fft"]) < tol


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("l1,l2,Lm", [(0, 0, 0), (2, 0, 2), (2, 2, 0), (2, 2, 2), (0, 2, 2), (1, 1, 0), (1, 1, 2),
                                       (3, 1, 2), (4, 2, 2)])
def test_sugiyama_vs_oracle(l1, l2, Lm, form):
    n, nb, dk = 32, 4, 0.012
    g, r, ora = _oracle(l1, l2, Lm)
    dt, prec, tol = FORMS[form]
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dt, observer=P.OBS)
    bins = cn.kbins(0.0, dk, nb)
    res = pl.measure_sugiyama(d, P.dev(g), P.dev(r), bins, l1, l2, Lm, precision=prec)
    for k in ("raw", "shot", "value"):
        assert P.rel(P.host(res[k]), ora[k]) < tol, k


def test_sugiyama_b000_equals_triposh_b000():
    n, nb, dk = 32, 4, 0.012
    g, r = P._cat(19, 30_000, 150_000)
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=L.F64, observer=P.OBS)
    bins = cn.kbins(0.0, dk, nb)
    gd, rd = P.dev(g), P.dev(r)
    for noise in ("analytic", "fft"):
        sg = pl.measure_sugiyama(d, gd, rd, bins, 0, 0, 0, noise=noise)
        tp = pl.measure_bk(d, gd, rd, bins, estimator=L.EST_TRIPOSH, ell=0, noise=noise)
        cfg, _ = tp["plan"].configs()
        S = {k: P.host(sg[k]) for k in ("raw", "shot", "value")}
        for t, (i, j, _) in enumerate(cfg):
            for k in ("raw", "shot", "value"):
                ref = P.host(tp[k])[t]
                assert abs(S[k][i, j] - ref) <= 1e-10 * abs(ref), (noise, k, i, j)
                assert abs(S[k][j, i] - ref) <= 1e-10 * abs(ref), (noise, k, j, i)


def test_sugiyama_many_shells_bf16_vs_fp64():
    """64^3, 10 shells (20 leg fields: 210 shell-pair slots, 7 pair tiles)."""
    n, nb, dk = 64, 10, 0.01
    g, r = P._cat(29, 40_000, 200_000)
    bins = cn.kbins(0.0, dk, nb)
    out = {}
    for form in ("f64", "bf16"):
        dt, prec, _ = FORMS[form]
        d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dt, observer=P.OBS)
        res = pl.measure_sugiyama(d, P.dev(g), P.dev(r), bins, 2, 2, 2, precision=prec)
        out[form] = {k: P.host(res[k]).copy() for k in ("raw", "shot", "value")}
    for k in ("raw", "shot", "value"):
        assert np.all(np.isfinite(out["f64"][k]))
        assert P.rel(out["bf16"][k], out["f64"][k]) < 1e-3, k


def test_sugiyama_argument_errors():
    d = cn.mesh_desc(32, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=P.OBS)
    bins = cn.kbins(0.0, 0.012, 4)
    with pytest.raises(L.CnpcError):
        pl.SugiPlan(d, bins, 2, 2, 6, L.PREC_F32)  # L outside {0, 2, 4}
    with pytest.raises(L.CnpcError):
        pl.SugiPlan(d, bins, 2, 1, 2, L.PREC_F32)  # odd l1 + l2
    with pytest.raises(L.CnpcError):
        pl.SugiPlan(d, bins, 4, 0, 2, L.PREC_F32)  # triangle rule
    with pytest.raises(L.CnpcError):
        pl.SugiPlan(d, cn.kbins(0.0, 0.005, 30), 2, 2, 0, L.PREC_BF16X3)  # too many shells for BF16
    sc = pl.Scratch()
    plan = pl.bispec_plan(d, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F32, sc)
    z = torch.zeros(16, dtype=torch.float64, device="cuda")
    st = L.lib.cnpc_sugiyama(plan.handle, L.ptr(z), None, None, L.ptr(z), L.ptr(z), L.ptr(z), L.ptr(z), L.ptr(z),
                             128, None)
    assert st != 0 and "cnpc_sugi_plan_create" in L.last_error()
