"""FFT-method shot noise of the TripoSH BB_l0l against the FP64 oracle,
through the C ABI.

The i = j != k term is the exact pair sum of P = F_l N* - s_l over the shell
pairs (no thin-shell step); the raw estimator and the other noise terms are
those of the analytic path, which must stay unchanged.  Bars: FP64 1e-10,
FP32 1e-5, split BF16 1e-3 (relative to the largest magnitude).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
from oracle.pipeline import MeshConfig, measure_bk  # noqa: E402
import test_gpu_parity as P  # noqa: E402

_ORACLE = {}


def _oracle(ell, n, nb, dk, seed):
    key = (ell, n, nb, dk, seed)
    if key not in _ORACLE:
        g, r = P._cat(seed, 30_000, 150_000)
        cfg = MeshConfig(1000.0, n, L.TSC, True, P.OBS)
        _ORACLE[key] = (g, r, measure_bk(g, None, r, None, cfg, dk, nb, ells=tuple(sorted({0, ell})),
                                         scoccimarro=(), triposh=(ell,), fft_noise=True))
    return _ORACLE[key]


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("ell", [0, 2])
def test_triposh_fft_noise_vs_oracle(ell, form):
    n, nb, dk = 32, 4, 0.012
    g, r, ora = _oracle(ell, n, nb, dk, 7)
    dt, prec, tol = {"f64": (L.F64, L.PREC_F64, 1e-10), "f32": (L.F32, L.PREC_F32, 1e-5),
                     "bf16": (L.F32, L.PREC_BF16X3, 1e-3)}[form]
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dt, observer=P.OBS)
    bins = cn.kbins(0.0, dk, nb)
    gd, rd = P.dev(g), P.dev(r)
    fft = pl.measure_bk(d, gd, rd, bins, estimator=L.EST_TRIPOSH, ell=ell, precision=prec, noise="fft")
    ana = pl.measure_bk(d, gd, rd, bins, estimator=L.EST_TRIPOSH, ell=ell, precision=prec)
    key = f"BB{ell}0{ell}"
    assert P.rel(P.host(fft["raw"]), ora[f"{key}_raw"]) < tol
    assert P.rel(P.host(fft["shot"]), ora[f"{key}_shot_fft"]) < tol
    assert P.rel(P.host(fft["value"]), ora[f"{key}_fft"]) < tol
    assert P.rel(P.host(ana["shot"]), ora[f"{key}_shot"]) < tol
    # the two methods differ by the thin-shell step only
    assert not np.array_equal(P.host(fft["shot"]), P.host(ana["shot"]))


def test_triposh_fft_noise_many_shells_bf16():
    """64^3, 10 shells (55 pairs: two pair tiles), split BF16 against FP64."""
    n, nb, dk = 64, 10, 0.01
    g, r = P._cat(61, 40_000, 200_000)
    bins = cn.kbins(0.0, dk, nb)
    out = {}
    for form, dt, prec in (("f64", L.F64, L.PREC_F64), ("bf16", L.F32, L.PREC_BF16X3)):
        d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dt, observer=P.OBS)
        res = pl.measure_bk(d, P.dev(g), P.dev(r), bins, estimator=L.EST_TRIPOSH, ell=2, precision=prec,
                            noise="fft")
        out[form] = {k: P.host(res[k]).copy() for k in ("raw", "shot", "value")}
    for k in ("raw", "shot", "value"):
        assert np.all(np.isfinite(out["f64"][k]))
        assert P.rel(out["bf16"][k], out["f64"][k]) < 1e-3, k


def test_fft_noise_rejects_scoccimarro_plans():
    d = cn.mesh_desc(32, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=P.OBS)
    bins = cn.kbins(0.0, 0.012, 4)
    sc = pl.Scratch()
    plan = pl.bispec_plan(d, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F32, sc)
    assert L.lib.cnpc_bispec_indicator_bytes(plan.handle) == 0
    with pytest.raises(ValueError):
        plan.indicators(sc)
    g, r = P._cat(7, 3000, 15000)
    with pytest.raises(ValueError):
        pl.measure_bk(d, P.dev(g), P.dev(r), bins, estimator=L.EST_SCOCCIMARRO, noise="fft")
