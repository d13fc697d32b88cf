"""The library's own batch (cnpc_batch_*) against the single-catalog calls.

An eager native batch must reproduce measure_pk_bk catalog by catalog
(identical kernels and order: P_l and B_0 equal to FP64 rounding of the
reductions, mode counts implied); the captured graph, replayed several times
with unrelated eager work and synchronisations in between, must reproduce the
eager batch every time; argument errors come back as CnpcError."""

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
import test_gpu_parity as P  # noqa: E402


def _setup(n=64, dtype=L.F32, prec=L.PREC_BF16X3, ncat=5, nb=6, dk=0.01):
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dtype, observer=P.OBS)
    bins = cn.kbins(0.0, dk, nb)
    sc = pl.Scratch()
    plan = pl.bispec_plan(d, bins, L.EST_SCOCCIMARRO, 0, prec, sc)
    cats = [P._cat(71 + 3 * k, 8_000 * (k + 1), 50_000 * (k + 1)) for k in range(ncat)]
    cats = [(P.dev(g), P.dev(r)) for g, r in cats]
    return d, bins, sc, plan, cats


def _outs(cats, plan, nb):
    return [{"pk": torch.full((9, nb), float("nan"), dtype=torch.float64, device="cuda"),
             "bk": torch.full((3, plan.nconf), float("nan"), dtype=torch.float64, device="cuda")} for _ in cats]


@pytest.mark.parametrize("nstreams,ells", [(1, (0, 2, 4)), (3, (0, 2, 4)), (2, (0,)), (2, (0, 2))])
def test_native_batch_matches_single_calls(nstreams, ells):
    d, bins, sc, plan, cats = _setup()
    ref = []
    for g, r in cats:
        o = pl.measure_pk_bk(d, g, r, bins, plan, ells=ells, scratch=sc)
        ref.append((P.host(o["pk"]).copy(), P.host(o["bk"]).copy()))
    nb = bins.nbins
    b = pl.NativeBatch(d, bins, plan, ells=ells, nstreams=nstreams,
                       max_ngal=max(g.shape[1] for g, _ in cats), max_nran=max(r.shape[1] for _, r in cats))
    outs = _outs(cats, plan, nb)
    b.run(cats, outs)
    torch.cuda.synchronize()
    for (pk, bk), o in zip(ref, outs):
        assert P.rel(P.host(o["pk"]), pk) < 1e-12
        assert P.rel(P.host(o["bk"]), bk) < 1e-12


@pytest.mark.parametrize("ells", [(0, 2, 4), (0, 2)])
def test_native_batch_256_matches_single_calls(ells):
    """At 256^3 with the benchmark's bins the batch takes its own routes: the
    de-aliased mesh handed to the Y_lm bases pass as z half spectra, the row
    coefficient table formed once, the shells' c2r inside the contraction;
    the single calls store the real mesh and form their own table.  Same
    transforms in differently compiled kernels, so the results agree to FP32
    rounding (a mistake in the hand-over would show at order one)."""
    d, bins, sc, plan, cats = _setup(n=256, ncat=2, nb=20)
    ref = []
    for g, r in cats:
        o = pl.measure_pk_bk(d, g, r, bins, plan, ells=ells, scratch=sc)
        ref.append((P.host(o["pk"]).copy(), P.host(o["bk"]).copy()))
    b = pl.NativeBatch(d, bins, plan, ells=ells, nstreams=2,
                       max_ngal=max(g.shape[1] for g, _ in cats), max_nran=max(r.shape[1] for _, r in cats))
    outs = _outs(cats, plan, bins.nbins)
    b.run(cats, outs)
    torch.cuda.synchronize()
    for (pk, bk), o in zip(ref, outs):
        assert P.rel(P.host(o["pk"]), pk) < 1e-6
        assert P.rel(P.host(o["bk"]), bk) < 1e-6


@pytest.mark.parametrize("dtype,prec", [(L.F32, L.PREC_BF16X3), (L.F64, L.PREC_F64)])
def test_native_batch_graph_replays(dtype, prec):
    d, bins, sc, plan, cats = _setup(dtype=dtype, prec=prec, ncat=4)
    nb = bins.nbins
    mx = (max(g.shape[1] for g, _ in cats), max(r.shape[1] for _, r in cats))
    b = pl.NativeBatch(d, bins, plan, nstreams=2, max_ngal=mx[0], max_nran=mx[1])
    outs = _outs(cats, plan, nb)
    b.run(cats, outs)
    torch.cuda.synchronize()
    eager = [(P.host(o["pk"]).copy(), P.host(o["bk"]).copy()) for o in outs]
    b.capture(cats, outs)
    for rep in range(3):
        for o in outs:
            o["pk"].fill_(float("nan"))
            o["bk"].fill_(float("nan"))
        # unrelated eager library work between replays
        pl.measure_pk(d, cats[0][0], cats[0][1], bins, ells=(0,), scratch=sc)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for (pk, bk), o in zip(eager, outs):
            assert P.rel(P.host(o["pk"]), pk) < 1e-12, rep
            assert P.rel(P.host(o["bk"]), bk) < 1e-12, rep


def test_native_batch_errors():
    d, bins, sc, plan, cats = _setup(ncat=2)
    nb = bins.nbins
    with pytest.raises(L.CnpcError):
        pl.NativeBatch(d, bins, plan, ells=(2, 4), nstreams=2, max_ngal=10, max_nran=10)  # no l = 0
    with pytest.raises(L.CnpcError):
        pl.NativeBatch(d, bins, plan, nstreams=0, max_ngal=10, max_nran=10)
    tri = pl.bispec_plan(d, bins, L.EST_TRIPOSH, 0, L.PREC_BF16X3, sc)
    with pytest.raises(L.CnpcError):
        pl.NativeBatch(d, bins, tri, nstreams=2, max_ngal=10, max_nran=10)
    b = pl.NativeBatch(d, bins, plan, nstreams=2, max_ngal=10, max_nran=10)
    with pytest.raises(L.CnpcError):
        b.run(cats, _outs(cats, plan, nb))  # catalogs above the maxima
    with pytest.raises(L.CnpcError):
        b.replay()  # nothing captured
