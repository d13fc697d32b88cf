"""cnpc_bin_pk_noalloc (no workspace argument, static device scratch) against
cnpc_bin_pk (caller workspace) through the C ABI: two calls in a row on the
same device, the second with fewer bins and products, each compared with the
workspace form (FP64 shell means and self terms within 1e-12 of their largest
value, mode counts bit-exact); and the host-side rejection of a binning larger
than the static scratch."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402


def _spectra(band, count, seed, dtype):
    g = torch.Generator().manual_seed(seed)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    return [torch.randn((4 * band ** 3, 2), generator=g, dtype=torch.float64).to(tdt).cuda()
            for _ in range(count)]


def _norms():
    nm = np.zeros(L.NORMS_LEN)
    nm[L.NORM_ALPHA], nm[L.NORM_I22], nm[L.NORM_N0], nm[L.NORM_SBAR] = 0.1, 3.0, 0.2, 5.0
    nm[L.NORM_SBARLM] = 5.0  # Sbar_0^0 (real part)
    nm[L.NORM_SBARLM + 2] = 1.5  # Sbar_2^0
    return torch.from_numpy(nm).cuda()


def _call(noalloc, d, bins, band, pairs, self_ells, norms):
    nb = bins.nbins
    npairs, nself = len(pairs), len(self_ells)
    means = torch.full((max(npairs, 1), nb), np.nan, dtype=torch.float64, device="cuda")
    selft = torch.full((max(nself, 1), nb), np.nan, dtype=torch.float64, device="cuda")
    nmodes = torch.full((nb,), -1, dtype=torch.int64, device="cuda")
    keff = torch.full((nb,), np.nan, dtype=torch.float64, device="cuda")
    pa = (C.c_void_p * max(npairs, 1))(*[L.ptr(a) for a, _ in pairs])
    pb = (C.c_void_p * max(npairs, 1))(*[L.ptr(b) for _, b in pairs])
    se = (C.c_int32 * max(nself, 1))(*self_ells)
    s = L.stream_handle()
    if noalloc:
        st = L.lib.cnpc_bin_pk_noalloc(C.byref(d), C.byref(bins), band, npairs, pa, pb, nself, se, L.ptr(norms),
                                       L.ptr(means), L.ptr(selft), L.ptr(nmodes), L.ptr(keff), s)
    else:
        ws = torch.empty(L.lib.cnpc_bin_pk_workspace_size(C.byref(bins), npairs, nself), dtype=torch.uint8,
                         device="cuda")
        st = L.lib.cnpc_bin_pk(C.byref(d), C.byref(bins), band, npairs, pa, pb, nself, se, L.ptr(norms),
                               L.ptr(means), L.ptr(selft), L.ptr(nmodes), L.ptr(keff), L.ptr(ws), ws.numel(), s)
    L.check(st)
    torch.cuda.synchronize()
    return (means[:npairs].cpu().numpy(), selft[:nself].cpu().numpy(), nmodes.cpu().numpy(),
            keff.cpu().numpy())


def _close(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b))) / scale < 1e-12


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
def test_noalloc_matches_workspace_form_twice(dtype):
    n, box, band = 64, 1000.0, 32
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype,
                     observer=(-866.0254037844386,) * 3)
    norms = _norms()
    spec = _spectra(band, 6, 5 + dtype, dtype)
    cases = [
        (cn.kbins(0.0, 0.01, 20), [(spec[0], spec[1]), (spec[2], spec[3]), (spec[4], spec[5])], [0, 2]),
        (cn.kbins(0.005, 0.02, 6), [(spec[1], spec[0])], [0]),  # smaller: fewer bins and products
    ]
    for bins, pairs, self_ells in cases:
        ref = _call(False, d, bins, band, pairs, self_ells, norms)
        got = _call(True, d, bins, band, pairs, self_ells, norms)
        assert np.array_equal(got[2], ref[2])
        assert _close(got[0], ref[0]) and _close(got[1], ref[1]) and _close(got[3], ref[3])
        assert not np.isnan(got[0]).any() and not np.isnan(got[1]).any()


def test_noalloc_rejects_binning_beyond_scratch():
    d = cn.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32)
    bins = cn.kbins(0.0, 0.001, 129)
    st = L.lib.cnpc_bin_pk_noalloc(C.byref(d), C.byref(bins), 128, 16, None, None, 4, None, None, None, None,
                                   None, None, None)
    assert st != 0 and "static scratch" in L.last_error()
