"""GPU parity of every hot-path step against the FP64 oracle (through the C ABI).

Bars: FP64 paths within 1e-10 (relative to the largest magnitude), FP32 paths
within 1e-5, integer outputs (cell patterns, mode counts, triangle counts)
bit-exact.  Sizes span several 16^3 paint tiles and FFT column tiles.
"""

import ctypes as C
import math

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
from oracle import mesh as oms  # noqa: E402
from oracle import spectra as osp  # noqa: E402
from oracle.catalog import catalog_norms  # noqa: E402
from oracle.pipeline import MeshConfig, measure_bk, measure_pk  # noqa: E402
import synthcat  # noqa: E402

OBS = synthcat.observer_position()
TOL = {L.F64: 1e-10, L.F32: 1e-5}


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------- FFT -----
@pytest.mark.parametrize("dtype", [L.F32, L.F64])
@pytest.mark.parametrize("n", [16, 32, 64, 128, 256])
def test_fft_full_r2c_c2r(n, dtype):
    rng = np.random.default_rng(n)
    x = rng.normal(size=(2, n, n, n))
    d = cn.mesh_desc(n, 100.0, dtype=dtype)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    xin = dev(x, tdt)
    spec = torch.empty((2, n, n, n // 2, 2), dtype=tdt, device="cuda")
    L.check(L.lib.cnpc_fft_r2c(C.byref(d), 2, 0, L.ptr(xin), L.ptr(spec), None, 0, L.stream_handle()))
    ref = np.fft.rfftn(x, axes=(1, 2, 3))[..., : n // 2]
    got = host(spec)
    got = got[..., 0] + 1j * got[..., 1]
    assert rel(got, ref) < 10 * TOL[dtype]
    # inverse: unnormalised, kz = N/2 plane absent
    back = torch.empty_like(xin)
    L.check(L.lib.cnpc_fft_c2r(C.byref(d), 2, 0, L.ptr(spec), L.ptr(back), None, 0, L.stream_handle()))
    full = np.fft.rfftn(x, axes=(1, 2, 3))
    full[..., n // 2] = 0.0
    refb = np.fft.irfftn(full, s=(n, n, n), axes=(1, 2, 3)) * n ** 3
    assert rel(host(back), refb) < 10 * TOL[dtype]


@pytest.mark.parametrize("dtype", [L.F32, L.F64])
@pytest.mark.parametrize("n,band", [(32, 8), (64, 16), (64, 32), (128, 32), (256, 32)])
def test_fft_band_r2c_c2r(n, band, dtype):
    rng = np.random.default_rng(n + band)
    x = rng.normal(size=(3, n, n, n))
    d = cn.mesh_desc(n, 100.0, dtype=dtype)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    xin = dev(x, tdt)
    spec = torch.empty((3, 2 * band, 2 * band, band, 2), dtype=tdt, device="cuda")
    wsb = L.lib.cnpc_fft_workspace_size(C.byref(d), 3, band)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.check(L.lib.cnpc_fft_r2c(C.byref(d), 3, band, L.ptr(xin), L.ptr(spec), L.ptr(ws), wsb,
                               L.stream_handle()))
    full = np.fft.rfftn(x, axes=(1, 2, 3))
    idx = np.r_[0:band, n - band:n]
    ref = full[:, idx][:, :, idx][..., :band]
    got = host(spec)
    got = got[..., 0] + 1j * got[..., 1]
    assert rel(got, ref) < 10 * TOL[dtype]
    back = torch.empty_like(xin)
    L.check(L.lib.cnpc_fft_c2r(C.byref(d), 3, band, L.ptr(spec), L.ptr(back), L.ptr(ws), wsb,
                               L.stream_handle()))
    trunc = np.zeros_like(full)
    trunc[np.ix_(range(3), idx, idx, range(band))] = ref
    # inverse band transforms read the unpaired n = -M rows as zero
    trunc[:, n - band] = 0.0
    trunc[:, :, n - band] = 0.0
    refb = np.fft.irfftn(trunc, s=(n, n, n), axes=(1, 2, 3)) * n ** 3
    assert rel(host(back), refb) < 10 * TOL[dtype]


def test_fft_band_512():
    """Band transforms at 512^3 (register column and z-row passes, N = 16 x 32)."""
    n, band = 512, 64
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1, n, n, n)).astype(np.float32)
    d = cn.mesh_desc(n, 100.0, dtype=L.F32)
    xin = dev(x)
    spec = torch.empty((1, 2 * band, 2 * band, band, 2), dtype=torch.float32, device="cuda")
    wsb = L.lib.cnpc_fft_workspace_size(C.byref(d), 1, band)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.check(L.lib.cnpc_fft_r2c(C.byref(d), 1, band, L.ptr(xin), L.ptr(spec), L.ptr(ws), wsb,
                               L.stream_handle()))
    full = np.fft.rfftn(x[0].astype(np.float64))
    idx = np.r_[0:band, n - band:n]
    ref = full[idx][:, idx][..., :band]
    del full
    got = host(spec)[0]
    got = got[..., 0] + 1j * got[..., 1]
    assert rel(got, ref) < 10 * TOL[L.F32]
    back = torch.empty_like(xin)
    L.check(L.lib.cnpc_fft_c2r(C.byref(d), 1, band, L.ptr(spec), L.ptr(back), L.ptr(ws), wsb,
                               L.stream_handle()))
    trunc = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    trunc[np.ix_(idx, idx, range(band))] = ref
    trunc[n - band] = 0.0
    trunc[:, n - band] = 0.0
    refb = np.fft.irfftn(trunc, s=(n, n, n), axes=(0, 1, 2)) * n ** 3
    assert rel(host(back)[0], refb) < 10 * TOL[L.F32]


# -------------------------------------------------------------- paint -----
def _tiny(seed, ng, nr, weights=False):
    g, gw, r, rw = synthcat.tiny_catalog(ng, nr, seed=seed, weights=weights)
    return g, gw, r, rw


@pytest.mark.parametrize("dtype", [L.F32, L.F64])
@pytest.mark.parametrize("assign,interlace", [(L.CIC, False), (L.CIC, True), (L.TSC, False), (L.TSC, True)])
@pytest.mark.parametrize("weights", [False, True])
def test_paint_and_norms(assign, interlace, weights, dtype):
    n, box = 32, 500.0
    g, gw, r, rw = _tiny(3 + assign, 3000, 20000, weights)
    d = cn.mesh_desc(n, box, assign=assign, interlace=interlace, dtype=dtype, observer=OBS)
    gt, rt = dev(g), dev(r)
    gwt = dev(gw) if weights else None
    rwt = dev(rw) if weights else None
    norms, gs, rs = pl.catalog_norms(d, gt, rt, gwt, rwt)
    ora = catalog_norms(g, gw, r, rw, box, OBS, (0, 2, 4))
    hn = host(norms)
    for k, v in ((L.NORM_ALPHA, ora.alpha), (L.NORM_NBAR, ora.nbar), (L.NORM_I22, ora.I22),
                 (L.NORM_I33, ora.I33), (L.NORM_N0, ora.N0), (L.NORM_SBAR, ora.Sbar)):
        assert math.isclose(hn[k], v, rel_tol=1e-12)
    q = 0
    for l in (0, 2, 4):
        for m in range(0, l + 1):
            sb = ora.Sbar_lm[(l, m)]
            assert abs(complex(hn[L.NORM_SBARLM + 2 * q], hn[L.NORM_SBARLM + 2 * q + 1]) - sb) < 1e-9 * max(1, abs(ora.Sbar))
            q += 1
    delta, nmesh = pl.paint(d, gt, rt, norms, gwt, rwt, noise=True)
    od, onm = oms.paint_fkp(g, gw, r, rw, ora.alpha, n, assign, interlace, noise=True)
    hd, hnm = host(delta), host(nmesh)
    for ph in range(2 if interlace else 1):
        assert rel(hd[ph], od[ph]) < 20 * TOL[dtype]
        assert rel(hnm[ph], onm[ph]) < 20 * TOL[dtype]


@pytest.mark.parametrize("case", ["dense128", "sparse256_weighted", "one_tile256"])
def test_paint_bucketed_sort(case):
    """Meshes with several tile buckets: bucket step, tile step (LDS runs and
    the per-particle path for chunks spanning many buckets), against the oracle."""
    rng = np.random.default_rng(21)
    if case == "dense128":
        n, box, assign, interlace, dtype = 128, 1000.0, L.TSC, True, L.F32
        g = synthcat.lognormal_catalog(200_000, box, 5)
        r = synthcat.random_catalog(1_000_000, 6)
        gw = rw = None
    elif case == "sparse256_weighted":
        n, box, assign, interlace, dtype = 256, 1000.0, L.CIC, False, L.F64
        g, gw, r, rw = _tiny(8, 5000, 30000, True)
    else:
        n, box, assign, interlace, dtype = 256, 1000.0, L.TSC, True, L.F32
        # every particle inside one 16^3-node tile (plus its stencil halo)
        g = (rng.integers(0, 2 ** 32 // 16, size=(3, 20000), dtype=np.uint32) + np.uint32(2 ** 31))
        r = (rng.integers(0, 2 ** 32 // 16, size=(3, 90000), dtype=np.uint32) + np.uint32(2 ** 31))
        gw = rw = None
    g, r = np.ascontiguousarray(g), np.ascontiguousarray(r)
    d = cn.mesh_desc(n, box, assign=assign, interlace=interlace, dtype=dtype, observer=OBS)
    gwt = dev(gw) if gw is not None else None
    rwt = dev(rw) if rw is not None else None
    norms, _, _ = pl.catalog_norms(d, dev(g), dev(r), gwt, rwt)
    delta, nmesh = pl.paint(d, dev(g), dev(r), norms, gwt, rwt, noise=True)
    alpha = float(host(norms)[L.NORM_ALPHA])
    od, onm = oms.paint_fkp(g, gw, r, rw, alpha, n, assign, interlace, noise=True)
    hd, hnm = host(delta), host(nmesh)
    for ph in range(2 if interlace else 1):
        assert rel(hd[ph], od[ph]) < 20 * TOL[dtype]
        assert rel(hnm[ph], onm[ph]) < 20 * TOL[dtype]


@pytest.mark.parametrize("n,weights,dtype", [(32, False, L.F32), (32, True, L.F64), (128, False, L.F32)])
def test_paint_fkp_matches_separate_calls(n, weights, dtype):
    """The fused entry point (sums, tile counts and, with several tile buckets,
    the first sort step in one pass) against cnpc_catalog_sums + cnpc_norms +
    cnpc_paint: bit-identical with one bucket or with the fused sort switched
    off, within a few ulp (summation order) otherwise."""
    if n == 32:
        g, gw, r, rw = _tiny(12, 4000, 30000, weights)
    else:
        g = synthcat.lognormal_catalog(100_000, 1000.0, 13)
        r = synthcat.random_catalog(500_000, 14)
        gw = rw = None
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dtype, observer=OBS)
    gt, rt = dev(g), dev(r)
    gwt = dev(gw) if gw is not None else None
    rwt = dev(rw) if rw is not None else None
    norms, gs, rs = pl.catalog_norms(d, gt, rt, gwt, rwt)
    delta, nmesh = pl.paint(d, gt, rt, norms, gwt, rwt, noise=True)
    norms2, delta2, nmesh2, gs2, rs2 = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True)
    if n == 32:  # one tile bucket: the sums pass of the separate calls
        for a, b in ((norms, norms2), (gs, gs2), (rs, rs2), (delta, delta2), (nmesh, nmesh2)):
            assert np.array_equal(host(a), host(b))
    else:
        # several buckets: sums taken in the bucket pass (another summation
        # order: a few ulp), meshes equal up to the rounding of alpha
        for a, b in ((norms, norms2), (gs, gs2), (rs, rs2)):
            assert np.allclose(host(a), host(b), rtol=1e-14, atol=1e-14 * np.max(np.abs(host(b))))
        for a, b in ((delta, delta2), (nmesh, nmesh2)):
            assert rel(host(a), host(b)) < (1e-14 if dtype == L.F64 else 1e-6)
        from paper_2605_04864_amd import autotune
        autotune.set_knobs({"sort_fused": 1})
        try:
            norms3, delta3, nmesh3, gs3, rs3 = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True)
        finally:
            autotune.reset_knobs()
        for a, b in ((norms, norms3), (gs, gs3), (rs, rs3), (delta, delta3), (nmesh, nmesh3)):
            assert np.array_equal(host(a), host(b))
        # l = 0 sums in the bucket pass, Y_lm sums in their own pass: the sums of
        # that pass equal the separate calls' bit for bit
        autotune.set_knobs({"sort_fused": 2})
        try:
            norms4, delta4, nmesh4, gs4, rs4 = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True)
        finally:
            autotune.reset_knobs()
        for a, b in ((norms, norms4), (gs, gs4), (rs, rs4), (delta, delta4), (nmesh, nmesh4)):
            assert np.array_equal(host(a), host(b))
    # l = 0 sums only: the same w sums, meshes and l = 0 normalisations, zero Y_lm sums
    norms0, delta0, nmesh0, gs0, rs0 = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True, sums_lmax=0)
    for a, b in ((delta2, delta0), (nmesh2, nmesh0)):
        assert np.array_equal(host(a), host(b))
    assert np.array_equal(host(gs2)[:5], host(gs0)[:5]) and not np.any(host(gs0)[5:])
    assert np.array_equal(host(rs2)[:5], host(rs0)[:5]) and not np.any(host(rs0)[5:])
    assert np.array_equal(host(norms2)[:L.NORM_SBARLM + 2], host(norms0)[:L.NORM_SBARLM + 2])


_OVF = {}


def _overflow_case(weights):
    """Catalogs that overflow the fixed-capacity bucket regions of the fused
    bucket pass on a 256^3 mesh (64 buckets of 4^3 tiles): half of each catalog
    in one bucket's 64^3-node cube, a fifth in one 16^3-node tile, the rest
    uniform (a survey footprint inside its box is of this kind).  The oracle's
    norms and meshes are cached per weighting."""
    if weights in _OVF:
        return _OVF[weights]
    rng = np.random.default_rng(31)

    def mix(n, tile_corner):
        a, b = n // 2, n // 5
        cube = rng.integers(0, 2 ** 30, size=(3, a), dtype=np.uint32)
        tile = rng.integers(0, 2 ** 28, size=(3, b), dtype=np.uint32) + np.uint32(tile_corner)
        rest = rng.integers(0, 2 ** 32, size=(3, n - a - b), dtype=np.uint32)
        p = np.concatenate([cube, tile, rest], axis=1)
        return np.ascontiguousarray(p[:, rng.permutation(n)])

    g, r = mix(150_000, 2 ** 31), mix(600_000, 3 * 2 ** 30)
    gw = rng.uniform(0.5, 1.5, g.shape[1]).astype(np.float32) if weights else None
    rw = rng.uniform(0.5, 1.5, r.shape[1]).astype(np.float32) if weights else None
    ora = catalog_norms(g, gw, r, rw, 1000.0, OBS, (0, 2, 4))
    od, onm = oms.paint_fkp(g, gw, r, rw, ora.alpha, 256, L.TSC, True, noise=True)
    _OVF[weights] = (g, gw, r, rw, ora, od, onm)
    return _OVF[weights]


@pytest.mark.parametrize("bucket,sums_lmax,weights", [(0, 0, False), (0, 4, False), (1, 0, False),
                                                      (2, 4, False), (3, 0, False), (0, 4, True)])
def test_paint_fkp_bucket_overflow(bucket, sums_lmax, weights):
    """The fused bucket pass when most records overflow their bucket regions
    (the tile pass then walks the overflow records with one slot per record),
    for every bucket-pass shape: meshes against the oracle's and against the
    separate calls, whose sort has no capacity limit."""
    from paper_2605_04864_amd import autotune
    g, gw, r, rw, ora, od, onm = _overflow_case(weights)
    d = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32, observer=OBS)
    gt, rt = dev(g), dev(r)
    gwt = dev(gw) if weights else None
    rwt = dev(rw) if weights else None
    autotune.set_knobs({"bucket": bucket})
    try:
        norms, delta, nmesh, _, _ = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True, sums_lmax=sums_lmax)
        hn, hd, hnm = host(norms), host(delta), host(nmesh)
    finally:
        autotune.reset_knobs()
    for k, v in ((L.NORM_ALPHA, ora.alpha), (L.NORM_I22, ora.I22), (L.NORM_N0, ora.N0)):
        assert math.isclose(hn[k], v, rel_tol=1e-12)
    for ph in range(2):
        assert rel(hd[ph], od[ph]) < 20 * TOL[L.F32]
        assert rel(hnm[ph], onm[ph]) < 20 * TOL[L.F32]
    norms2, _, _ = pl.catalog_norms(d, gt, rt, gwt, rwt)
    delta2, nmesh2 = pl.paint(d, gt, rt, norms2, gwt, rwt, noise=True)
    assert rel(hd, host(delta2)) < 1e-6
    assert rel(hnm, host(nmesh2)) < 1e-6


def test_paint_f32_256_position_grid():
    """Unit-weight FP32 painting on 256^3 takes the positions truncated to a
    2^-17 cell grid inside their 16^3 tile (8-byte sort records): its meshes
    match the oracle painting the truncated positions to the fixed-point
    rounding, several times closer than the oracle painting the exact ones;
    the FP64 path keeps the exact positions."""
    rng = np.random.default_rng(17)
    n, box = 256, 1000.0
    g = rng.integers(0, 2 ** 32, size=(3, 20000), dtype=np.uint32)
    r = rng.integers(0, 2 ** 32, size=(3, 60000), dtype=np.uint32)
    down = (32 - 8) - 17  # fraction bits below the grid
    trunc = np.uint32(0xFFFFFFFF ^ ((1 << down) - 1))
    gt, rt = g & trunc, r & trunc
    out = {}
    for dt in (L.F32, L.F64):
        d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dt, observer=OBS)
        norms, _, _ = pl.catalog_norms(d, dev(g), dev(r))
        delta, _ = pl.paint(d, dev(g), dev(r), norms, noise=False)
        out[dt] = (float(host(norms)[L.NORM_ALPHA]), host(delta))
    alpha = out[L.F64][0]
    exact, _ = oms.paint_fkp(g, None, r, None, alpha, n, L.TSC, True, noise=False)
    grid, _ = oms.paint_fkp(gt, None, rt, None, alpha, n, L.TSC, True, noise=False)
    for ph in range(2):
        e_grid = rel(out[L.F32][1][ph], grid[ph])
        e_exact = rel(out[L.F32][1][ph], exact[ph])
        assert e_grid < 1e-6 and e_exact > 3 * e_grid, (e_grid, e_exact)
        e64_exact = rel(out[L.F64][1][ph], exact[ph])
        e64_grid = rel(out[L.F64][1][ph], grid[ph])
        assert e64_exact < 20 * TOL[L.F64] and e64_grid > 100 * e64_exact, (e64_exact, e64_grid)


def test_paint_single_particle_cells_bit_exact():
    n, box = 32, 100.0
    rng = np.random.default_rng(9)
    for assign in (L.CIC, L.TSC):
        for trial in range(20):
            p = rng.integers(0, 2 ** 32, size=(3, 1), dtype=np.uint32)
            if trial == 0:
                p[:] = np.uint32(2 ** 32 - 1)  # wraps at the upper edge
            if trial == 1:
                p[:] = np.uint32(0)
            r = rng.integers(0, 2 ** 32, size=(3, 1), dtype=np.uint32)
            d = cn.mesh_desc(n, box, assign=assign, interlace=True, dtype=L.F64, observer=OBS)
            norms, _, _ = pl.catalog_norms(d, dev(p), dev(r))
            delta, _ = pl.paint(d, dev(p), dev(r), norms, noise=False)
            ga = oms.paint(p, None, n, assign, 0.0)
            gb = oms.paint(p, None, n, assign, 0.5)
            hd = host(delta)
            ra = oms.paint(r, None, n, assign, 0.0)
            rb = oms.paint(r, None, n, assign, 0.5)
            # alpha = 1: delta = g - r; compare the supports of g alone via exactness of sums
            assert np.array_equal(np.abs(hd[0] - (ga - ra)) < 1e-12, np.ones_like(ga, bool))
            assert np.array_equal(np.abs(hd[1] - (gb - rb)) < 1e-12, np.ones_like(gb, bool))


# --------------------------------------------------------------- ylm ------
@pytest.mark.parametrize("dtype", [L.F32, L.F64])
@pytest.mark.parametrize("ell", [1, 2, 3, 4])
def test_ylm_fields(ell, dtype):
    from oracle.ylm import ylm_racah
    n, box = 16, 300.0
    d = cn.mesh_desc(n, box, dtype=dtype, observer=OBS)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    delta = np.random.default_rng(ell).normal(size=(n, n, n))
    out = torch.empty((2 * ell + 1, n, n, n), dtype=tdt, device="cuda")
    L.check(L.lib.cnpc_ylm_fields(C.byref(d), ell, L.ptr(dev(delta, tdt)), L.ptr(out), L.stream_handle()))
    rvec = osp.line_of_sight(n, box, OBS)
    got = host(out)
    refs = [delta * ylm_racah(ell, 0, rvec).real]
    for m in range(1, ell + 1):
        y = ylm_racah(ell, m, rvec)
        refs += [delta * y.real, delta * y.imag]
    for f, ref in enumerate(refs):
        assert rel(got[f], ref) < 10 * TOL[dtype] + 1e-7 * (dtype == L.F32)


YLM_LOS = (0.3, -0.5, 0.812403840463596)


# FP32 at N = 256 (bands of whole 16-column tiles) writes the z-power bases and
# forms the fields in the y pass; FP32 at N = 64 forms them in the z pass from
# bases held in registers; FP64 and N = 128 take one transform per field
@pytest.mark.parametrize("n,band,dtype,ells,los", [
    (64, 16, L.F64, (2, 4), None), (128, 32, L.F32, (2, 4), None), (256, 32, L.F32, (2, 4), None),
    (256, 64, L.F64, (2, 4), None), (64, 16, L.F32, (1, 2, 3, 4), None), (256, 64, L.F32, (2, 4), None),
    (256, 128, L.F32, (2, 4), None), (64, 16, L.F32, (1, 2, 3, 4), YLM_LOS),
    (256, 32, L.F32, (2, 4), YLM_LOS), (256, 32, L.F32, (1, 2, 3, 4), None), (256, 16, L.F32, (2,), None)])
def test_ylm_r2c_band(n, band, dtype, ells, los):
    """Y_lm-weighted band transforms (fused prologue z-pass + band column
    passes) against numpy FFTs of the explicitly weighted fields."""
    from oracle.ylm import ylm_racah
    box = 1000.0
    d = cn.mesh_desc(n, box, dtype=dtype, observer=OBS, los=los)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    delta = np.random.default_rng(n + band).normal(size=(n, n, n))
    got = pl.ylm_spectra(d, band, ells, dev(delta, tdt))
    rvec = osp.line_of_sight(n, box, OBS, los)
    idx = np.r_[0:band, n - band:n]
    for ell in ells:
        fields = [ylm_racah(ell, 0, rvec).real]
        for m in range(1, ell + 1):
            y = ylm_racah(ell, m, rvec)
            fields += [y.real, y.imag]
        g = host(got[ell])
        for f, w in enumerate(fields):
            ref = np.fft.rfftn(delta * w)[np.ix_(idx, idx, range(band))]
            gf = g[f, ..., 0] + 1j * g[f, ..., 1]
            assert rel(gf.reshape(ref.shape), ref) < 20 * TOL[dtype], (ell, f)


# ---------------------------------------------------------- power ---------
def _cat(seed, ng, nr):
    g = synthcat.lognormal_catalog(ng, 1000.0, seed)
    r = synthcat.random_catalog(nr, seed + 1)
    return g, r


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
@pytest.mark.parametrize("n,assign,interlace", [(32, L.CIC, False), (64, L.TSC, True)])
def test_measure_pk_vs_oracle(n, assign, interlace, dtype):
    box = 1000.0
    g, r = _cat(100 + n, 40_000, 200_000)
    kN = math.pi * n / box
    nb = int(kN // 0.01) - 1
    bins = cn.kbins(0.0, 0.01, nb)
    d = cn.mesh_desc(n, box, assign=assign, interlace=interlace, dtype=dtype, observer=OBS)
    res = pl.measure_pk(d, dev(g), dev(r), bins, ells=(0, 2, 4), modified=True)
    cfg = MeshConfig(box, n, assign, interlace, OBS)
    ora = measure_pk(g, None, r, None, cfg, 0.0, 0.01, nb, ells=(0, 2, 4), modified=True)
    assert np.array_equal(host(res["nmodes"]), ora["nmodes"])
    assert rel(host(res["k_eff"]), ora["k_eff"]) < 1e-12
    for key in ("P0", "P2", "P4", "P22", "P42", "P44", "P4b", "P6b", "P8b"):
        assert rel(host(res[key]), ora[key]) < TOL[dtype], key


# ---------------------------------------------------------- bispectrum ----
@pytest.mark.parametrize("dtype", [L.F64, L.F32])
@pytest.mark.parametrize("est,ell", [(L.EST_SCOCCIMARRO, 0), (L.EST_SCOCCIMARRO, 2),
                                     (L.EST_TRIPOSH, 0), (L.EST_TRIPOSH, 2)])
def test_measure_bk_vs_oracle(est, ell, dtype):
    n, box = 32, 1000.0
    nb, dk = 4, 0.012
    g, r = _cat(7, 30_000, 150_000)
    bins = cn.kbins(0.0, dk, nb)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype, observer=OBS)
    res = pl.measure_bk(d, dev(g), dev(r), bins, estimator=est, ell=ell)
    cfg = MeshConfig(box, n, L.TSC, True, OBS)
    sc = (ell,) if est == L.EST_SCOCCIMARRO else ()
    tr = (ell,) if est == L.EST_TRIPOSH else ()
    ora = measure_bk(g, None, r, None, cfg, dk, nb, ells=tuple(sorted({0, ell})), scoccimarro=sc, triposh=tr)
    plan = res["plan"]
    ijk, ntri = plan.configs()
    if est == L.EST_SCOCCIMARRO:
        key = f"B{ell}"
        assert [tuple(c) for c in ijk] == [tuple(c) for c in ora[f"{key}_configs"]]
        assert np.array_equal(ntri, ora[f"{key}_ntri"])
    else:
        key = f"BB{ell}0{ell}"
        assert [tuple(c[:2]) for c in ijk] == [tuple(c) for c in ora[f"{key}_pairs"]]
    tol = TOL[dtype]
    assert rel(host(res["raw"]), ora[f"{key}_raw"]) < tol
    assert rel(host(res["shot"]), ora[f"{key}_shot"]) < tol
    assert rel(host(res["value"]), ora[key]) < tol


@pytest.mark.parametrize("est,ell", [(L.EST_SCOCCIMARRO, 0), (L.EST_SCOCCIMARRO, 2), (L.EST_TRIPOSH, 2)])
def test_measure_bk_split_bf16_vs_oracle(est, ell):
    """Split-BF16 MFMA contraction: within 1e-3 of the FP64 oracle."""
    n, box = 32, 1000.0
    nb, dk = 4, 0.012
    g, r = _cat(7, 30_000, 150_000)
    bins = cn.kbins(0.0, dk, nb)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=OBS)
    res = pl.measure_bk(d, dev(g), dev(r), bins, estimator=est, ell=ell, precision=L.PREC_BF16X3)
    cfg = MeshConfig(box, n, L.TSC, True, OBS)
    sc = (ell,) if est == L.EST_SCOCCIMARRO else ()
    tr = (ell,) if est == L.EST_TRIPOSH else ()
    ora = measure_bk(g, None, r, None, cfg, dk, nb, ells=tuple(sorted({0, ell})), scoccimarro=sc, triposh=tr)
    key = f"B{ell}" if est == L.EST_SCOCCIMARRO else f"BB{ell}0{ell}"
    assert rel(host(res["raw"]), ora[f"{key}_raw"]) < 1e-3
    assert rel(host(res["value"]), ora[key]) < 1e-3


@pytest.mark.parametrize("est,ell,prec", [(L.EST_SCOCCIMARRO, 0, L.PREC_F64), (L.EST_SCOCCIMARRO, 2, L.PREC_BF16X3),
                                          (L.EST_TRIPOSH, 2, L.PREC_F64), (L.EST_TRIPOSH, 0, L.PREC_BF16X3)])
def test_measure_bk_reduced_grid_vs_oracle(est, ell, prec):
    """Shell fields on a 32^3 contraction grid for a 64^3 mesh (k_max far below
    Nyquist) against the oracle's sum over the full 64^3 mesh."""
    n, box = 64, 1000.0
    nb, dk = 4, 0.012
    g, r = _cat(11, 40_000, 200_000)
    bins = cn.kbins(0.0, dk, nb)
    dtype = L.F64 if prec == L.PREC_F64 else L.F32
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype, observer=OBS)
    res = pl.measure_bk(d, dev(g), dev(r), bins, estimator=est, ell=ell, precision=prec)
    plan = res["plan"]
    assert plan.grid == 32
    cfg = MeshConfig(box, n, L.TSC, True, OBS)
    sc = (ell,) if est == L.EST_SCOCCIMARRO else ()
    tr = (ell,) if est == L.EST_TRIPOSH else ()
    ora = measure_bk(g, None, r, None, cfg, dk, nb, ells=tuple(sorted({0, ell})), scoccimarro=sc, triposh=tr)
    key = f"B{ell}" if est == L.EST_SCOCCIMARRO else f"BB{ell}0{ell}"
    if est == L.EST_SCOCCIMARRO:
        ijk, ntri = plan.configs()
        assert np.array_equal(ntri, ora[f"{key}_ntri"])
    tol = TOL[L.F64] if prec == L.PREC_F64 else 1e-3
    assert rel(host(res["raw"]), ora[f"{key}_raw"]) < tol
    assert rel(host(res["value"]), ora[key]) < tol


_STAGED_SKIP = pytest.mark.skip(reason="the staged batch mode (painting and spectra on separate streams) was "
                                        "removed: never faster than the round-robin batch, and capturing it "
                                        "crashed the process at the end of the capture (cause not found)")


@pytest.mark.parametrize("nstreams,staged", [(1, False), (3, False), pytest.param(2, True, marks=_STAGED_SKIP),
                                             pytest.param(1, True, marks=_STAGED_SKIP)])
def test_graph_replay_matches_eager(nstreams, staged):
    """The batch captured as one graph (catalogs spread over nstreams streams)
    gives the eager single-stream results on every replay."""
    n, box = 32, 1000.0
    bins = cn.kbins(0.0, 0.012, 4)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=OBS)
    cats = [_cat(21 + 2 * k, 10_000 * (k + 1), 60_000 * (k + 1)) for k in range(4)]
    cats = [(dev(g), dev(r)) for g, r in cats]
    sc = pl.Scratch()
    plan = pl.bispec_plan(d, bins, L.EST_SCOCCIMARRO, 0, L.PREC_F32, sc)
    outs = [{"pk": torch.empty((9, 4), dtype=torch.float64, device="cuda"),
             "bk": torch.empty((3, plan.nconf), dtype=torch.float64, device="cuda")} for _ in cats]
    for (g, r), o in zip(cats, outs):
        pl.measure_pk_bk(d, g, r, bins, plan, scratch=sc, out=o)
    assert not staged
    batch = pl.Batch(nstreams)

    def step():
        batch.run(d, cats, bins, plan, outs)

    eager = [(host(o["pk"]).copy(), host(o["bk"]).copy()) for o in outs]
    step()  # eager multi-stream pass: scratch buffers reach their size
    torch.cuda.synchronize()
    for (pk, bk), o in zip(eager, outs):
        assert rel(host(o["pk"]), pk) < 1e-5
        assert rel(host(o["bk"]), bk) < 1e-5
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for o in outs:
            o["pk"].zero_()
            o["bk"].zero_()
        graph.replay()
        torch.cuda.synchronize()
        for (pk, bk), o in zip(eager, outs):
            assert rel(host(o["pk"]), pk) < 1e-5
            assert rel(host(o["bk"]), bk) < 1e-5
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays


@pytest.mark.parametrize("weights,dtype,band", [(False, L.F32, 32), (True, L.F32, 16), (True, L.F64, 32),
                                                (False, L.F64, 64)])
def test_paint_deinterlace_matches_two_steps(weights, dtype, band):
    """cnpc_paint_deinterlace (tile sums taken inside the z passes of the
    de-interlacing transforms) against cnpc_paint_fkp + cnpc_deinterlace of
    delta (band spectrum and delta_int) and of N (band spectrum), every band
    slot included."""
    n = 256
    if weights:
        g, gw, r, rw = _tiny(15, 60000, 300000, True)
    else:
        g = synthcat.lognormal_catalog(300_000, 1000.0, 17)
        r = synthcat.random_catalog(10 * g.shape[1], 18)
        gw = rw = None
    d = cn.mesh_desc(n, 1000.0, assign=L.TSC, interlace=True, dtype=dtype, observer=OBS)
    gt, rt = dev(g), dev(r)
    gwt = dev(gw) if gw is not None else None
    rwt = dev(rw) if rw is not None else None
    sc = pl.Scratch()
    norms, delta, nmesh, gs, rs = pl.paint_fkp(d, gt, rt, gwt, rwt, noise=True, scratch=sc)
    D, dint = pl.deinterlace(d, band, delta, want_real=True, scratch=sc)
    DN, _ = pl.deinterlace(d, band, nmesh, want_real=False, scratch=sc)
    norms2, D2, dint2, DN2, gs2, rs2 = pl.paint_deinterlace(d, band, gt, rt, gwt, rwt, scratch=sc)
    assert np.allclose(host(norms2), host(norms), rtol=1e-14, atol=0)
    tol = 1e-12 if dtype == L.F64 else 2e-6
    for a, b in ((D2, D), (dint2, dint), (DN2, DN)):
        assert rel(host(a), host(b)) < tol
