"""Full-size cases of the benchmark configurations, through the C ABI.

* c1 (64^3 CIC, 2e5 + 2e6 particles, plain FP64): P_0, P_2, P_4 against the
  FP64 oracle on the whole catalog, 1e-10; mode counts bit-exact.
* c2 (256^3 TSC + interlacing, 5e6 + 2.5e7): the FP32 path against the FP64
  path (pinned to the oracle at small sizes) within 1e-5 for every P_l,
  P_ll' and P_lb; mode counts and k_eff against the oracle's binning.
* c3 (256^3, 2e6 + 2e7, 20 bins): Scoccimarro B_0, B_2 and TripoSH B_202 in
  FP32 (1e-5) and split BF16 (1e-3) against FP64; triangle counts of sampled
  configurations against the oracle's indicator-field triple sums, bit-exact.
* c4 (the benchmark's batch): its smallest, median and largest mocks through
  the library's batch runner and its captured graph, FP32 / split BF16
  against the FP64 path (1e-5 / 1e-3), configurations, N_T and mode counts.
* c5 (512^3, L = 2000, 3e7 + 3e8, 40 bins of 0.005): TripoSH B_202 in split
  BF16 (1e-3) and FP32 (1e-5) against FP64; mode counts and k_eff against the
  oracle's binning of the whole 512^3 grid.

Catalogs follow the benchmark recipe (seed 1000 * config for galaxies, + 1 for
randoms).
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
from oracle import bispectrum as obk  # noqa: E402
from oracle import spectra as osp  # noqa: E402
from oracle.pipeline import MeshConfig, measure_pk  # noqa: E402
import synthcat  # noqa: E402
import test_gpu_parity as P  # noqa: E402

OBS = synthcat.observer_position()
_CATS = {}


def catalogs(config):
    """Host and device catalogs of a configuration (kept for the module)."""
    if config not in _CATS:
        spec = synthcat.config_spec(config)
        g = synthcat.lognormal_catalog(spec.ngal, spec.boxsize, 1000 * config)
        r = synthcat.random_catalog(spec.nran, 1000 * config + 1)
        _CATS[config] = (spec, g, r, P.dev(g), P.dev(r))
    return _CATS[config]


def descs(spec):
    return {dt: cn.mesh_desc(spec.nmesh, spec.boxsize, assign=spec.assign, interlace=spec.interlace,
                             dtype=dt, observer=OBS) for dt in (L.F32, L.F64)}


def test_c1_full_fp64_vs_oracle():
    spec, g, r, gd, rd = catalogs(1)
    d = descs(spec)[L.F64]
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    res = pl.measure_pk(d, gd, rd, bins, ells=(0, 2, 4))
    cfg = MeshConfig(spec.boxsize, spec.nmesh, spec.assign, spec.interlace, OBS)
    ora = measure_pk(g, None, r, None, cfg, 0.0, spec.dk, spec.nbins, ells=(0, 2, 4))
    assert np.array_equal(P.host(res["nmodes"]), ora["nmodes"])
    for key in ("P0", "P2", "P4"):
        assert P.rel(P.host(res[key]), ora[key]) < 1e-10, key


def test_c2_full_fp32_vs_fp64():
    spec, g, r, gd, rd = catalogs(2)
    ds = descs(spec)
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    r64 = pl.measure_pk(ds[L.F64], gd, rd, bins, ells=(0, 2, 4), modified=True)
    r32 = pl.measure_pk(ds[L.F32], gd, rd, bins, ells=(0, 2, 4), modified=True)
    ob = osp.Bins(0.0, spec.dk, spec.nbins, spec.boxsize, spec.nmesh)
    assert np.array_equal(P.host(r64["nmodes"]), ob.counts())
    assert np.array_equal(P.host(r32["nmodes"]), ob.counts())
    assert P.rel(P.host(r64["k_eff"]), ob.k_eff()) < 1e-12
    for key in pl.PK_ROWS:
        assert P.rel(P.host(r32[key]), P.host(r64[key])) < 1e-5, key


@pytest.mark.parametrize("name,est,ell", [("B0", L.EST_SCOCCIMARRO, 0), ("B2", L.EST_SCOCCIMARRO, 2),
                                          ("B202", L.EST_TRIPOSH, 2)])
def test_c3_full_precisions(name, est, ell):
    spec, g, r, gd, rd = catalogs(3)
    ds = descs(spec)
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    out = {}
    for form, dt, prec in (("f64", L.F64, L.PREC_F64), ("f32", L.F32, L.PREC_F32),
                           ("bf16", L.F32, L.PREC_BF16X3)):
        res = pl.measure_bk(ds[dt], gd, rd, bins, estimator=est, ell=ell, precision=prec)
        out[form] = {k: P.host(res[k]).copy() for k in ("raw", "value")}
        if est == L.EST_SCOCCIMARRO:
            out[form]["configs"] = res["plan"].configs()
    for k in ("raw", "value"):
        assert P.rel(out["f32"][k], out["f64"][k]) < 1e-5, k
        assert P.rel(out["bf16"][k], out["f64"][k]) < 1e-3, k
    if est == L.EST_SCOCCIMARRO:
        ijk, nt = out["f64"]["configs"]
        for form in ("f32", "bf16"):
            assert np.array_equal(out[form]["configs"][0], ijk)
            assert np.array_equal(out[form]["configs"][1], nt)
        if ell == 0:
            # sampled configurations: N_T from the oracle's indicator fields on
            # the 256^3 mesh (one triple sum each)
            ob = osp.Bins(0.0, spec.dk, spec.nbins, spec.boxsize, spec.nmesh)
            shells = ob.shell_index()
            pick = [0, len(ijk) // 3, len(ijk) // 2, len(ijk) - 1]
            need = sorted({int(b) for q in pick for b in ijk[q]})
            ind = {b: obk.indicator_field(shells, b) for b in need}
            n3 = float(spec.nmesh) ** 3
            for q in pick:
                i, j, k = (int(x) for x in ijk[q])
                ref = obk.triple_sum(ind[i], ind[j], ind[k]) / n3
                assert abs(ref - round(ref)) < 1e-6
                assert int(nt[q]) == int(round(ref)), (i, j, k)


def test_c5_full_triposh_precisions():
    spec, g, r, gd, rd = catalogs(5)
    ds = descs(spec)
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    out = {}
    for form, dt, prec in (("f64", L.F64, L.PREC_F64), ("f32", L.F32, L.PREC_F32),
                           ("bf16", L.F32, L.PREC_BF16X3)):
        res = pl.measure_bk(ds[dt], gd, rd, bins, estimator=L.EST_TRIPOSH, ell=2, precision=prec)
        out[form] = {k: P.host(res[k]).copy() for k in ("raw", "value")}
        assert res["plan"].nconf == spec.nbins * (spec.nbins + 1) // 2
    for k in ("raw", "value"):
        assert np.all(np.isfinite(out["f64"][k]))
        assert P.rel(out["f32"][k], out["f64"][k]) < 1e-5, k
        assert P.rel(out["bf16"][k], out["f64"][k]) < 1e-3, k


def test_c5_mode_counts_vs_oracle():
    """c5's binning at full size (512^3, L = 2000, 40 bins of 0.005): the mode
    counts of every bin bit-exact and k_eff within 1e-12 against the oracle's
    integer-n^2 binning of the whole grid (FP32 and FP64 paths)."""
    spec, g, r, gd, rd = catalogs(5)
    ds = descs(spec)
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    ob = osp.Bins(0.0, spec.dk, spec.nbins, spec.boxsize, spec.nmesh)
    counts, keff = ob.counts(), ob.k_eff()
    for dt in (L.F32, L.F64):
        res = pl.measure_pk(ds[dt], gd, rd, bins, ells=(0, 2))
        assert np.array_equal(P.host(res["nmodes"]), counts)
        assert P.rel(P.host(res["k_eff"]), keff) < 1e-12


def test_c4_batch_graph_vs_fp64():
    """c4 in the launch configuration of the benchmark: mocks of the c4 size
    distribution (its smallest, median and largest: 1.0e6, 2.5e6, 7.9e6
    galaxies with 10x randoms, the benchmark's seeds) through the library's
    batch runner, captured as one graph and replayed, in FP32 fields with the
    split-BF16 contraction; against the plain FP64 path mock by mock (P_l
    within 1e-5, B_0 within 1e-3), identical configurations and N_T, and the
    mode counts of the oracle's binning."""
    sizes = synthcat.mock_sizes_c4(64)
    pick = [63, 4, 54]
    mocks = []
    for k in pick:
        ng = int(sizes[k])
        g = synthcat.lognormal_catalog(ng, 1000.0, 4000 + 2 * k)
        r = synthcat.random_catalog(10 * ng, 4000 + 2 * k + 1)
        mocks.append((P.dev(g), P.dev(r)))
        del g, r
    bins = cn.kbins(0.0, 0.01, 20)
    d32 = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=OBS)
    d64 = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F64, observer=OBS)
    sc, sc64 = pl.Scratch(), pl.Scratch()
    plan32 = pl.bispec_plan(d32, bins, L.EST_SCOCCIMARRO, 0, L.PREC_BF16X3, sc)
    plan64 = pl.bispec_plan(d64, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F64, sc64)
    c32, c64 = plan32.configs(), plan64.configs()
    assert np.array_equal(c32[0], c64[0]) and np.array_equal(c32[1], c64[1])
    batch = pl.NativeBatch(d32, bins, plan32, nstreams=2, max_ngal=max(int(g.shape[1]) for g, _ in mocks),
                           max_nran=max(int(r.shape[1]) for _, r in mocks))
    outs = [{"pk": torch.empty((9, 20), dtype=torch.float64, device="cuda"),
             "bk": torch.empty((3, plan32.nconf), dtype=torch.float64, device="cuda")} for _ in mocks]
    batch.capture(mocks, outs)
    batch.replay()
    torch.cuda.synchronize()
    ob = osp.Bins(0.0, 0.01, 20, 1000.0, 256)
    for (g, r), o in zip(mocks, outs):
        ref = pl.measure_pk_bk(d64, g, r, bins, plan64, scratch=sc64)
        assert np.array_equal(P.host(ref["nmodes"]), ob.counts())
        for row in range(3):  # P_0, P_2, P_4
            assert P.rel(P.host(o["pk"][row]), P.host(ref["pk"][row])) < 1e-5, row
        for row in range(3):  # raw, shot, value
            assert P.rel(P.host(o["bk"][row]), P.host(ref["bk"][row])) < 1e-3, row
