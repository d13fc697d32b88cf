"""The library against stored FP64 oracle outputs at the benchmark's full sizes.

The fixtures ``tests/golden/oracle_c2.json``, ``oracle_c3.json`` and
``oracle_c4min.json`` were written by ``tests/golden/make_oracle_fixtures.py``,
which calls only the oracle.  Each test regenerates the seeded catalog, checks
its SHA-256 against the fixture (so a different catalog fails loudly instead of
comparing unrelated numbers), runs the library and compares element by element
with the relative error of reading R21 (max over bins of |X - X_oracle| over
max |X_oracle|, per multipole vector):

* FP64 path within 1e-10, FP32 fields with FP64 accumulators within 1e-5,
  split-BF16 contraction within 1e-3 (eqs. Hand17, Plnew, bi_sco, new_bispec);
* mode counts, configurations and triangle counts bit-exact.
c4min is the smallest mock of the 64-mock batch, run through the library's
batch runner and its captured graph as the benchmark runs it.
"""

import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
import synthcat  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
OBS = synthcat.observer_position()
TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-3}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def fixture(case):
    with open(os.path.join(GOLDEN, f"oracle_{case}.json")) as fh:
        fx = json.load(fh)
    if case in ("c2", "c3"):
        config = int(case[1])
        spec = synthcat.config_spec(config)
        g = synthcat.lognormal_catalog(spec.ngal, spec.boxsize, 1000 * config)
        r = synthcat.random_catalog(spec.nran, 1000 * config + 1)
    else:
        spec = synthcat.config_spec(4)
        sizes = synthcat.mock_sizes_c4(64)
        k = int(np.argmin(sizes))
        g = synthcat.lognormal_catalog(int(sizes[k]), spec.boxsize, 4000 + 2 * k)
        r = synthcat.random_catalog(10 * int(sizes[k]), 4000 + 2 * k + 1)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g).tobytes())
    h.update(np.ascontiguousarray(r).tobytes())
    assert h.hexdigest() == fx["catalog_sha256"], f"{case}: regenerated catalog differs from the fixture's"
    gd, rd = torch.from_numpy(g).cuda(), torch.from_numpy(r).cuda()
    return spec, fx, gd, rd


def desc(spec, dt):
    return cn.mesh_desc(spec.nmesh, spec.boxsize, assign=spec.assign, interlace=spec.interlace,
                        dtype=dt, observer=OBS)


@pytest.fixture(scope="module")
def c2():
    return fixture("c2")


@pytest.fixture(scope="module")
def c3():
    return fixture("c3")


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_c2_pk_vs_oracle(c2, form):
    spec, fx, gd, rd = c2
    dt = L.F64 if form == "f64" else L.F32
    res = pl.measure_pk(desc(spec, dt), gd, rd, cn.kbins(0.0, spec.dk, spec.nbins), ells=(0, 2, 4),
                        modified=True)
    assert list(host(res["nmodes"])) == fx["nmodes"]
    assert rel(host(res["k_eff"]), fx["k_eff"]) < 1e-12
    errs = {k: rel(host(res[k]), fx["pk"][k]) for k in pl.PK_ROWS}
    bad = {k: v for k, v in errs.items() if not v < TOL[form]}
    assert not bad, (form, errs)


@pytest.mark.parametrize("form", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("key,est,ell", [("B0", L.EST_SCOCCIMARRO, 0), ("B2", L.EST_SCOCCIMARRO, 2),
                                         ("BB202", L.EST_TRIPOSH, 2)])
def test_c3_bk_vs_oracle(c3, key, est, ell, form):
    spec, fx, gd, rd = c3
    dt = L.F64 if form == "f64" else L.F32
    prec = {"f64": L.PREC_F64, "f32": L.PREC_F32, "bf16": L.PREC_BF16X3}[form]
    res = pl.measure_bk(desc(spec, dt), gd, rd, cn.kbins(0.0, spec.dk, spec.nbins), estimator=est, ell=ell,
                        precision=prec)
    ref = fx[key]
    ijk, ntri = res["plan"].configs()
    if est == L.EST_SCOCCIMARRO:
        assert [list(map(int, c)) for c in ijk] == ref["configs"]
        assert [int(x) for x in ntri] == ref["ntri"]
    else:
        assert [list(map(int, c[:2])) for c in ijk] == ref["pairs"]
    raw = np.asarray(ref["raw"])
    shot = np.asarray(ref["shot"])
    errs = {"raw": rel(host(res["raw"]), raw), "shot": rel(host(res["shot"]), shot),
            "value": rel(host(res["value"]), raw - shot)}
    # the shot noise uses no contraction: FP32 bar even with the split-BF16 GEMM
    bars = {"raw": TOL[form], "shot": TOL["f32"] if form == "bf16" else TOL[form], "value": TOL[form]}
    assert all(errs[k] < bars[k] for k in errs), (key, form, errs)


def test_c4_smallest_mock_batch_graph_vs_oracle():
    spec, fx, gd, rd = fixture("c4min")
    bins = cn.kbins(0.0, spec.dk, spec.nbins)
    d32 = desc(spec, L.F32)
    sc = pl.Scratch()
    plan = pl.bispec_plan(d32, bins, L.EST_SCOCCIMARRO, 0, L.PREC_BF16X3, sc)
    ijk, ntri = plan.configs()
    assert [list(map(int, c)) for c in ijk] == fx["B0"]["configs"]
    assert [int(x) for x in ntri] == fx["B0"]["ntri"]
    batch = pl.NativeBatch(d32, bins, plan, nstreams=1, max_ngal=int(gd.shape[1]), max_nran=int(rd.shape[1]))
    out = [{"pk": torch.empty((9, spec.nbins), dtype=torch.float64, device="cuda"),
            "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device="cuda")}]
    batch.capture([(gd, rd)], out)
    batch.replay()
    pk, bk = host(out[0]["pk"]), host(out[0]["bk"])
    errs = {k: rel(pk[row], fx["pk"][k]) for row, k in enumerate(("P0", "P2", "P4"))}
    raw, shot = np.asarray(fx["B0"]["raw"]), np.asarray(fx["B0"]["shot"])
    errs.update({"B0 raw": rel(bk[0], raw), "B0 shot": rel(bk[1], shot), "B0": rel(bk[2], raw - shot)})
    bars = {"P0": TOL["f32"], "P2": TOL["f32"], "P4": TOL["f32"], "B0 raw": TOL["bf16"],
            "B0 shot": TOL["f32"], "B0": TOL["bf16"]}
    assert all(errs[k] < bars[k] for k in errs), errs
    # the plain FP64 path on the same mock
    d64 = desc(spec, L.F64)
    sc64 = pl.Scratch()
    plan64 = pl.bispec_plan(d64, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F64, sc64)
    ref = pl.measure_pk_bk(d64, gd, rd, bins, plan64, scratch=sc64)
    assert list(host(ref["nmodes"])) == fx["nmodes"]
    p64, b64 = host(ref["pk"]), host(ref["bk"])
    for row, k in enumerate(("P0", "P2", "P4")):
        assert rel(p64[row], fx["pk"][k]) < TOL["f64"], k
    assert rel(b64[0], raw) < TOL["f64"] and rel(b64[1], shot) < TOL["f64"]
    assert rel(b64[2], raw - shot) < TOL["f64"]
