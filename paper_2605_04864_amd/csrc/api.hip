// C ABI: host-side argument validation and dispatch (see include/cnpc.h).
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bispec.h"

namespace cnpc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

size_t lds_limit() {
  static std::mutex mu;
  static size_t cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  std::lock_guard<std::mutex> lk(mu);
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 65536;
    cache[dev] = (size_t)v;
  }
  return cache[dev];
}

static bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// ----------------------------------------------------------- kernel timer --
struct KTimer {
  uint32_t mask = 0;
  int used = 0;
  int open_cls = -1;
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
};
static KTimer g_kt;

void kt_begin(int c, hipStream_t s) {
  if (((g_kt.mask >> c) & 1u) && g_kt.used + 2 <= (int)g_kt.ev.size()) {
    (void)hipEventRecord(g_kt.ev[g_kt.used], s);
    g_kt.open_cls = c;
  }
}
void kt_end(int c, hipStream_t s) {
  if (g_kt.open_cls == c && g_kt.used + 2 <= (int)g_kt.ev.size()) {
    (void)hipEventRecord(g_kt.ev[g_kt.used + 1], s);
    g_kt.cls[g_kt.used / 2] = c;
    g_kt.used += 2;
    g_kt.open_cls = -1;
  }
}

// -------------------------------------------------------- tuning knobs --
static std::atomic<int> g_tune[CNPC_TUNE_COUNT];

int tune_value(int knob) {
  return knob >= 0 && knob < CNPC_TUNE_COUNT ? g_tune[knob].load(std::memory_order_relaxed) : 0;
}

cnpc_status check_desc(const cnpc_mesh_desc* d) {
  CNPC_REQUIRE(d != nullptr, "null mesh descriptor");
  CNPC_REQUIRE(pow2(d->n) && d->n >= 16 && d->n <= 1024, "n must be a power of two in [16, 1024] (got %d)", d->n);
  CNPC_REQUIRE(d->assign == CNPC_CIC || d->assign == CNPC_TSC, "assign must be CNPC_CIC or CNPC_TSC");
  CNPC_REQUIRE(d->interlace == 0 || d->interlace == 1, "interlace must be 0 or 1");
  CNPC_REQUIRE(d->dtype == CNPC_F32 || d->dtype == CNPC_F64, "dtype must be CNPC_F32 or CNPC_F64");
  CNPC_REQUIRE(std::isfinite(d->boxsize) && d->boxsize > 0, "boxsize must be positive");
  if (d->los_mode == CNPC_LOS_LOCAL) {
    bool inside = true;
    for (int i = 0; i < 3; ++i) {
      CNPC_REQUIRE(std::isfinite(d->observer[i]), "observer must be finite");
      if (d->observer[i] < 0 || d->observer[i] >= d->boxsize) inside = false;
    }
    CNPC_REQUIRE(!inside, "the observer must lie outside the box [0, L)^3");
  } else {
    CNPC_REQUIRE(d->los_mode == CNPC_LOS_GLOBAL, "los_mode must be CNPC_LOS_LOCAL or CNPC_LOS_GLOBAL");
    const double nrm = sqrt(d->los[0] * d->los[0] + d->los[1] * d->los[1] + d->los[2] * d->los[2]);
    CNPC_REQUIRE(fabs(nrm - 1.0) < 1e-6, "los must be a unit vector");
  }
  return CNPC_OK;
}

cnpc_status check_bins(const cnpc_mesh_desc* d, const cnpc_kbins* b) {
  CNPC_REQUIRE(b != nullptr, "null k-bins");
  CNPC_REQUIRE(b->nbins >= 1 && b->nbins <= MAX_BINS, "nbins must be in [1, %d]", MAX_BINS);
  CNPC_REQUIRE(std::isfinite(b->dk) && b->dk > 0, "dk must be positive");
  CNPC_REQUIRE(std::isfinite(b->kmin) && b->kmin >= 0, "kmin must be >= 0");
  const double kny = M_PI * d->n / d->boxsize;
  CNPC_REQUIRE(b->kmin + b->nbins * b->dk <= kny * (1 + 1e-12), "bins extend past the Nyquist wavenumber");
  return CNPC_OK;
}

void bin_thresholds(const cnpc_mesh_desc* d, const cnpc_kbins* b, int64_t* out) {
  // smallest integer n^2 at or above (edge / kf)^2; an edge whose square is
  // within a relative 1e-9 of an integer sits on it, so that the rounding of
  // dk and kf never moves a whole lattice shell across a half-open edge
  const double kf = 2.0 * M_PI / d->boxsize;
  for (int i = 0; i <= b->nbins; ++i) {
    const double x = (b->kmin + (double)i * b->dk) / kf;
    const double v = x * x;
    const double r = nearbyint(v);
    out[i] = (int64_t)(fabs(v - r) <= 1e-9 * fmax(1.0, v) ? r : ceil(v));
  }
}

}  // namespace cnpc

using namespace cnpc;

#define API_BEGIN clear_error()

extern "C" {

const char* cnpc_last_error(void) { return g_err.c_str(); }
const char* cnpc_version(void) { return "cnpc 0.1 (gfx950)"; }

cnpc_status cnpc_tune_set(int32_t knob, int32_t value) {
  API_BEGIN;
  CNPC_REQUIRE(knob >= 0 && knob < CNPC_TUNE_COUNT, "unknown tuning knob %d", knob);
  bool ok = value == 0;
  switch (knob) {
    case CNPC_TUNE_FFT_PASSES: ok = value == 0 || value == 1; break;
    case CNPC_TUNE_FFT_COL_W: ok = ok || (value > 0 && value <= 64 && (value & (value - 1)) == 0); break;
    case CNPC_TUNE_CONTRACT_KG:
    case CNPC_TUNE_SORT_PER: ok = ok || value == 1 || value == 2 || value == 4; break;
    case CNPC_TUNE_SORT_THREADS: ok = ok || value == 512 || value == 1024; break;
    case CNPC_TUNE_SORT_FUSED: ok = value >= 0 && value <= 2; break;
    case CNPC_TUNE_FOLD_FUSED: ok = value == 0 || value == 1; break;
    case CNPC_TUNE_BUCKET: ok = value >= 0 && value <= 3; break;
    case CNPC_TUNE_YLM_BASIS: ok = value == 0 || value == 1; break;
    case CNPC_TUNE_SHELL_FUSED: ok = value == 0 || value == 1; break;
  }
  CNPC_REQUIRE(ok, "value %d out of range for tuning knob %d", value, knob);
  g_tune[knob].store(value, std::memory_order_relaxed);
  return CNPC_OK;
}

int32_t cnpc_tune_get(int32_t knob) {
  return knob >= 0 && knob < CNPC_TUNE_COUNT ? g_tune[knob].load(std::memory_order_relaxed) : -1;
}

cnpc_status cnpc_ktimer_start(uint32_t class_mask, int32_t max_launches) {
  API_BEGIN;
  CNPC_REQUIRE(class_mask != 0 && (class_mask >> 16) == 0, "class mask must select classes 0..15");
  CNPC_REQUIRE(max_launches >= 1 && max_launches <= (1 << 20), "max_launches out of range");
  for (hipEvent_t e : g_kt.ev) (void)hipEventDestroy(e);
  g_kt.ev.assign(2 * (size_t)max_launches, nullptr);
  g_kt.cls.assign((size_t)max_launches, -1);
  for (auto& e : g_kt.ev) CNPC_HIP(hipEventCreate(&e));
  g_kt.used = 0;
  g_kt.open_cls = -1;
  g_kt.mask = class_mask;
  return CNPC_OK;
}

cnpc_status cnpc_ktimer_stop(double* ms_per_class, int64_t* launches_per_class) {
  API_BEGIN;
  double tot[16] = {0};
  int64_t cnt[16] = {0};
  cnpc_status st = CNPC_OK;
  for (int i = 0; i + 1 < g_kt.used; i += 2) {
    float ms = 0.f;
    if (hipEventSynchronize(g_kt.ev[i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, g_kt.ev[i], g_kt.ev[i + 1]) != hipSuccess) {
      set_error("kernel timer events failed");
      st = CNPC_EHIP;
      break;
    }
    const int c = g_kt.cls[i / 2];
    if (c >= 0 && c < 16) { tot[c] += ms; cnt[c]++; }
  }
  for (int c = 0; c < 16; ++c) {
    if (ms_per_class) ms_per_class[c] = tot[c];
    if (launches_per_class) launches_per_class[c] = cnt[c];
  }
  for (hipEvent_t e : g_kt.ev) (void)hipEventDestroy(e);
  g_kt.ev.clear();
  g_kt.cls.clear();
  g_kt.used = 0;
  g_kt.mask = 0;
  return st;
}

size_t cnpc_catalog_sums_workspace_size(void) { return (size_t)1024 * CNPC_SUMS_LEN * sizeof(double); }

cnpc_status cnpc_catalog_sums(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w, int64_t n,
                              double* sums, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(n >= 1 && n < ((int64_t)1 << 32), "particle count must be in [1, 2^32)");
  CNPC_REQUIRE(pos && sums && ws, "null pointer argument");
  return launch_catalog_sums(d, pos, w, n, sums, ws, ws_bytes, as_stream(stream));
}

cnpc_status cnpc_norms(const cnpc_mesh_desc* d, const double* gs, const double* rs, int64_t ngal,
                       double* norms, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(gs && rs && norms, "null pointer argument");
  CNPC_REQUIRE(ngal >= 1, "ngal must be positive");
  return launch_norms(d, gs, rs, ngal, norms, as_stream(stream));
}

size_t cnpc_paint_workspace_size(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran) {
  if (check_desc(d) != CNPC_OK) return 0;
  return paint_layout(d, ngal, nran, true).total;
}

cnpc_status cnpc_paint(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw, int64_t ngal,
                       const uint32_t* rpos, const float* rw, int64_t nran, const double* norms,
                       void* delta, void* noise, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(ngal >= 1 && ngal < ((int64_t)1 << 32), "ngal must be in [1, 2^32)");
  CNPC_REQUIRE(nran >= 1 && nran < ((int64_t)1 << 32), "nran must be in [1, 2^32)");
  CNPC_REQUIRE(gpos && rpos && norms && delta && ws, "null pointer argument");
  CNPC_REQUIRE((gw == nullptr) == (rw == nullptr), "give weights for both catalogs or for neither");
  return launch_paint(d, gpos, gw, ngal, rpos, rw, nran, norms, delta, noise, ws, ws_bytes,
                      as_stream(stream));
}

cnpc_status cnpc_paint_fkp(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw, int64_t ngal,
                           const uint32_t* rpos, const float* rw, int64_t nran, int32_t sums_lmax,
                           double* gal_sums, double* ran_sums, double* norms, void* delta, void* noise,
                           void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(sums_lmax == 0 || sums_lmax == 2 || sums_lmax == 4, "sums_lmax must be 0, 2 or 4");
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(ngal >= 1 && ngal < ((int64_t)1 << 32), "ngal must be in [1, 2^32)");
  CNPC_REQUIRE(nran >= 1 && nran < ((int64_t)1 << 32), "nran must be in [1, 2^32)");
  CNPC_REQUIRE(gpos && rpos && norms && delta && ws, "null pointer argument");
  CNPC_REQUIRE((gw == nullptr) == (rw == nullptr), "give weights for both catalogs or for neither");
  return launch_paint_fkp(d, gpos, gw, ngal, rpos, rw, nran, sums_lmax, gal_sums, ran_sums, norms, delta,
                          noise, ws, ws_bytes, as_stream(stream));
}

static cnpc_status check_band(const cnpc_mesh_desc* d, int band) {
  CNPC_REQUIRE(band == 0 || (pow2(band) && band >= 1 && band <= d->n / 2),
               "band must be 0 (full) or a power of two <= n/2 (got %d)", band);
  return CNPC_OK;
}

size_t cnpc_fft_workspace_size(const cnpc_mesh_desc* d, int32_t batch, int32_t band) {
  if (check_desc(d) != CNPC_OK || batch < 1) return 0;
  return fft_ws_elems(d->n, batch, band) * 2 * esize(d->dtype);
}

cnpc_status cnpc_fft_r2c(const cnpc_mesh_desc* d, int32_t batch, int32_t band, const void* in, void* out,
                         void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(batch >= 1, "batch must be positive");
  CNPC_REQUIRE(in && out && in != out, "in and out must be distinct non-null pointers");
  const size_t need = fft_ws_elems(d->n, batch, band) * 2 * esize(d->dtype);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) {
    set_error("fft workspace too small: need %zu bytes", need);
    return CNPC_EWORKSPACE;
  }
  if (d->dtype == CNPC_F64)
    return fft3d_r2c<double>(d->n, batch, band, (const double*)in, (cx<double>*)out, (cx<double>*)ws,
                             as_stream(stream));
  return fft3d_r2c<float>(d->n, batch, band, (const float*)in, (cx<float>*)out, (cx<float>*)ws,
                          as_stream(stream));
}

cnpc_status cnpc_fft_c2r(const cnpc_mesh_desc* d, int32_t batch, int32_t band, const void* in, void* out,
                         void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(batch >= 1, "batch must be positive");
  CNPC_REQUIRE(in && out && in != out, "in and out must be distinct non-null pointers");
  const size_t need = fft_ws_elems(d->n, batch, band) * 2 * esize(d->dtype);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) {
    set_error("fft workspace too small: need %zu bytes", need);
    return CNPC_EWORKSPACE;
  }
  if (d->dtype == CNPC_F64)
    return fft3d_c2r<double>(d->n, batch, band, (const cx<double>*)in, (double*)out, (cx<double>*)ws,
                             as_stream(stream));
  return fft3d_c2r<float>(d->n, batch, band, (const cx<float>*)in, (float*)out, (cx<float>*)ws,
                          as_stream(stream));
}

int32_t cnpc_band_for(const cnpc_mesh_desc* d, double kmax) {
  if (check_desc(d) != CNPC_OK || !(kmax > 0)) return 0;
  const double kf = 2.0 * M_PI / d->boxsize;
  int m = 1;
  while (m < d->n / 2 && (double)m * kf <= kmax) m <<= 1;
  return m;
}

size_t cnpc_deinterlace_workspace_size(const cnpc_mesh_desc* d) {
  if (check_desc(d) != CNPC_OK) return 0;
  return deinterlace_ws_max(d);
}

cnpc_status cnpc_deinterlace(const cnpc_mesh_desc* d, int32_t band, const void* meshes, void* spec_band,
                             void* delta_int, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(band >= 1, "band must be >= 1");
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(meshes && spec_band && ws, "null pointer argument");
  return launch_deinterlace(d, band, meshes, spec_band, delta_int, ws, ws_bytes, as_stream(stream));
}

size_t cnpc_paint_deinterlace_workspace_size(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, int32_t weighted,
                                             int32_t band) {
  if (check_desc(d) != CNPC_OK || band < 1 || ngal < 1 || nran < 1) return 0;
  return paint_deinterlace_ws_bytes(d, ngal, nran, weighted != 0, band);
}

cnpc_status cnpc_paint_deinterlace(const cnpc_mesh_desc* d, int32_t band, const uint32_t* gpos, const float* gw,
                                   int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran, int32_t sums_lmax,
                                   double* gal_sums, double* ran_sums, double* norms, void* spec_band,
                                   void* delta_int, void* noise_spec_band, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(band >= 1, "band must be >= 1");
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(gpos && rpos && norms && spec_band && delta_int && noise_spec_band && ws, "null pointer argument");
  CNPC_REQUIRE(ngal >= 1 && nran >= 1, "empty catalog");
  CNPC_REQUIRE(sums_lmax == 0 || sums_lmax == 2 || sums_lmax == 4, "sums_lmax must be 0, 2 or 4");
  if (!has_fold_zr2c(d)) {
    set_error("painting with de-interlacing needs an interlaced 256^3 mesh with the register FFT passes");
    return CNPC_EUNSUPPORTED;
  }
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  // without caller arrays the sums go to the painting workspace's sums slots
  const size_t off_sums = paint_layout(d, ngal, nran, gw || rw).off_sums;
  double* gs = gal_sums ? gal_sums : reinterpret_cast<double*>(w + off_sums);
  double* rs = ran_sums ? ran_sums : reinterpret_cast<double*>(w + off_sums) + CNPC_SUMS_LEN;
  return launch_paint_deinterlace(d, band, gpos, gw, ngal, rpos, rw, nran, sums_lmax, gs, rs, norms, spec_band,
                                  delta_int, noise_spec_band, ws, ws_bytes, as_stream(stream));
}

cnpc_status cnpc_ylm_fields(const cnpc_mesh_desc* d, int32_t ell, const void* delta, void* out,
                            void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(ell >= 0 && ell <= 4, "ell must be in [0, 4]");
  CNPC_REQUIRE(delta && out && delta != out, "delta and out must be distinct non-null pointers");
  return launch_ylm_fields(d, ell, delta, out, as_stream(stream));
}

size_t cnpc_ylm_r2c_workspace_size(const cnpc_mesh_desc* d, int32_t nfields, int32_t band) {
  if (check_desc(d) != CNPC_OK || nfields < 1 || band < 1) return 0;
  return ylm_r2c_ws_bytes(d, nfields, band);
}

cnpc_status cnpc_ylm_r2c(const cnpc_mesh_desc* d, int32_t band, int32_t nells, const int32_t* ells,
                         const void* delta, void* out, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(band >= 1, "band must be >= 1");
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(nells >= 1 && ells != nullptr, "need at least one multipole");
  for (int q = 0; q < nells; ++q) CNPC_REQUIRE(ells[q] >= 1 && ells[q] <= 4, "ells must be in [1, 4]");
  CNPC_REQUIRE(delta && out && ws, "null pointer argument");
  return launch_ylm_r2c(d, band, nells, ells, delta, out, ws, ws_bytes, as_stream(stream));
}

cnpc_status cnpc_assemble_F(const cnpc_mesh_desc* d, int32_t band, int32_t ell, const void* spec0,
                            const void* ylm, void* F_out, void* stream) {
  API_BEGIN;
  CNPC_TRY(check_desc(d));
  CNPC_REQUIRE(band >= 1, "band must be >= 1");
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(ell >= 0 && ell <= 4, "ell must be in [0, 4]");
  CNPC_REQUIRE(F_out != nullptr, "null output");
  CNPC_REQUIRE(ell == 0 ? spec0 != nullptr : ylm != nullptr, "missing input spectra");
  return launch_assemble(d, band, ell, spec0, ylm, F_out, as_stream(stream));
}

size_t cnpc_bin_pk_workspace_size(const cnpc_kbins* b, int32_t npairs, int32_t nself) {
  if (!b || b->nbins < 1) return 0;
  return bin_ws_doubles(b->nbins, npairs, nself) * sizeof(double);
}

static cnpc_status bin_pk_common(const cnpc_mesh_desc* d, const cnpc_kbins* b, int32_t band, int32_t npairs,
                                 const void* const* pa, const void* const* pb, uint32_t imag, int32_t nself,
                                 const int32_t* self_ells, const double* norms, double* means,
                                 double* selfterm, int64_t* nmodes, double* keff, void* ws, size_t ws_bytes,
                                 void* stream) {
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_bins(d, b));
  CNPC_REQUIRE(band >= 1, "band must be >= 1");
  CNPC_TRY(check_band(d, band));
  CNPC_REQUIRE(npairs >= 0 && npairs <= MAX_PAIRS, "npairs must be in [0, %d]", MAX_PAIRS);
  CNPC_REQUIRE(nself >= 0 && nself <= MAX_SELF, "nself must be in [0, %d]", MAX_SELF);
  CNPC_REQUIRE(nmodes != nullptr && ws != nullptr, "null pointer argument");
  CNPC_REQUIRE(npairs == 0 || (pa && pb && means), "pairs need pa, pb and means");
  for (int q = 0; q < npairs; ++q) CNPC_REQUIRE(pa[q] && pb[q], "null spectrum pointer in pair %d", q);
  if (nself) {
    CNPC_REQUIRE(self_ells && selfterm && norms, "self terms need self_ells, selfterm and norms");
    for (int q = 0; q < nself; ++q)
      CNPC_REQUIRE(self_ells[q] == 0 || self_ells[q] == 2 || self_ells[q] == 4, "self_ells must be 0, 2 or 4");
  }
  // every binned mode must be inside the band
  const double kf = 2.0 * M_PI / d->boxsize;
  CNPC_REQUIRE((double)band * kf > b->kmin + b->nbins * b->dk || band == d->n / 2,
               "band %d does not cover the bins (k_max / k_f = %.2f)", band,
               (b->kmin + b->nbins * b->dk) / kf);
  if (ws_bytes < bin_ws_doubles(b->nbins, npairs, nself) * sizeof(double)) {
    set_error("bin_pk workspace too small");
    return CNPC_EWORKSPACE;
  }
  int64_t thr[MAX_BINS + 1];
  bin_thresholds(d, b, thr);
  return launch_bin(d, thr, b->nbins, band, npairs, pa, pb, imag, nself, self_ells, norms, (double*)ws, means,
                    selfterm, nmodes, keff, as_stream(stream));
}

cnpc_status cnpc_bin_pk(const cnpc_mesh_desc* d, const cnpc_kbins* b, int32_t band, int32_t npairs,
                        const void* const* pa, const void* const* pb, int32_t nself,
                        const int32_t* self_ells, const double* norms, double* means, double* selfterm,
                        int64_t* nmodes, double* keff, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  return bin_pk_common(d, b, band, npairs, pa, pb, 0u, nself, self_ells, norms, means, selfterm, nmodes, keff,
                       ws, ws_bytes, stream);
}

// Allocation-free bin_pk.  Its FP64 shell accumulators live in `scratch`, a
// file-scope device array sized for the largest binning cnpc_bin_pk accepts;
// each device holds its own copy, whose address is looked up once per device
// with that device current and kept.  Host code only ever uses that address:
// the array's name is a host-side stand-in, not a device pointer.
constexpr size_t NOALLOC_BIN_DOUBLES = (size_t)MAX_BINS * (MAX_PAIRS + MAX_SELF + 1);
static __device__ __align__(256) double scratch[NOALLOC_BIN_DOUBLES];

static cnpc_status noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* addr[64] = {nullptr};
  int dev = 0;
  CNPC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index %d out of range", dev);
    return CNPC_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("device %d: no address for the bin_pk scratch array (%s)", dev, hipGetErrorString(e));
      return CNPC_EHIP;
    }
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return CNPC_OK;
}

cnpc_status cnpc_bin_pk_noalloc(const cnpc_mesh_desc* d, const cnpc_kbins* b, int32_t band, int32_t npairs,
                                const void* const* pa, const void* const* pb, int32_t nself,
                                const int32_t* self_ells, const double* norms, double* means,
                                double* selfterm, int64_t* nmodes, double* keff, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(b != nullptr, "null k-bins");
  CNPC_REQUIRE(b->nbins >= 1 && npairs >= 0 && nself >= 0, "nbins must be >= 1, npairs and nself >= 0");
  const size_t need = bin_ws_doubles(b->nbins, npairs, nself);
  CNPC_REQUIRE(need <= NOALLOC_BIN_DOUBLES,
               "bin_pk_noalloc: nbins * (npairs + nself + 1) = %zu exceeds the static scratch of %zu doubles",
               need, NOALLOC_BIN_DOUBLES);
  double* ws = nullptr;
  CNPC_TRY(noalloc_scratch(&ws));
  return bin_pk_common(d, b, band, npairs, pa, pb, 0u, nself, self_ells, norms, means, selfterm, nmodes, keff,
                       ws, NOALLOC_BIN_DOUBLES * sizeof(double), stream);
}

cnpc_status cnpc_bin_pk_im(const cnpc_mesh_desc* d, const cnpc_kbins* b, int32_t band, int32_t npairs,
                           const void* const* pa, const void* const* pb, double* means, int64_t* nmodes,
                           double* keff, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  const uint32_t all = npairs >= 32 ? 0xffffffffu : ((1u << (npairs > 0 ? npairs : 0)) - 1u);
  return bin_pk_common(d, b, band, npairs, pa, pb, all, 0, nullptr, nullptr, means, nullptr, nmodes, keff,
                       ws, ws_bytes, stream);
}

cnpc_status cnpc_pk_multipole(const cnpc_kbins* b, int32_t ell, const double* mean, const double* norms,
                              double* out, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(b && b->nbins >= 1 && b->nbins <= MAX_BINS, "bad bins");
  CNPC_REQUIRE(ell >= 0 && ell <= 8, "ell must be in [0, 8]");
  CNPC_REQUIRE(mean && norms && out, "null pointer argument");
  return launch_pk_multipole(b->nbins, ell, mean, norms, out, as_stream(stream));
}

cnpc_status cnpc_cross_norms(const double* norms_a, const double* norms_b, double* norms_out, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(norms_a && norms_b && norms_out, "null pointer argument");
  return launch_cross_norms(norms_a, norms_b, norms_out, as_stream(stream));
}

cnpc_status cnpc_pk_finalize(const cnpc_kbins* b, const double* m00, const double* m02, const double* m04,
                             const double* m22, const double* m42, const double* m44, const double* norms,
                             double* out, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(b && b->nbins >= 1 && b->nbins <= MAX_BINS, "bad bins");
  CNPC_REQUIRE(norms && out, "null pointer argument");
  return launch_pk_finalize(b->nbins, m00, m02, m04, m22, m42, m44, norms, out, as_stream(stream));
}

size_t cnpc_bispec_workspace_size(const cnpc_mesh_desc* d, const cnpc_kbins* b, int32_t est, int32_t ell) {
  if (check_desc(d) != CNPC_OK || check_bins(d, b) != CNPC_OK) return 0;
  return bispec_ws_bytes(d, b, est, ell);
}

cnpc_status cnpc_bispec_plan_create(cnpc_bispec_plan** plan, const cnpc_mesh_desc* d, const cnpc_kbins* b,
                                    int32_t est, int32_t ell, int32_t prec, void* ws, size_t ws_bytes,
                                    void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(plan != nullptr, "null plan pointer");
  *plan = nullptr;
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_bins(d, b));
  CNPC_REQUIRE(est == CNPC_EST_SCOCCIMARRO || est == CNPC_EST_TRIPOSH, "unknown estimator");
  CNPC_REQUIRE(ell == 0 || ell == 2 || ell == 4, "ell must be 0, 2 or 4");
  CNPC_REQUIRE(prec == CNPC_PREC_F64 || prec == CNPC_PREC_F32 || prec == CNPC_PREC_BF16X3, "unknown precision");
  CNPC_REQUIRE(!(prec == CNPC_PREC_F64 && d->dtype != CNPC_F64), "CNPC_PREC_F64 needs FP64 fields");
  CNPC_REQUIRE(!(prec != CNPC_PREC_F64 && d->dtype != CNPC_F32), "FP32 / split-BF16 contraction needs FP32 fields");
  CNPC_REQUIRE(b->kmin == 0.0, "bispectrum bins must start at k = 0 (closure on bin centres)");
  CNPC_REQUIRE(est == CNPC_EST_TRIPOSH || b->nbins <= MAX_COLS, "at most %d Scoccimarro shells", MAX_COLS);
  const double kny = M_PI * d->n / d->boxsize;
  if (est == CNPC_EST_TRIPOSH)
    CNPC_REQUIRE((2 * b->nbins - 1) * b->dk <= kny, "TripoSH shot noise needs bins up to 2 k_max below Nyquist");
  CNPC_REQUIRE(ws != nullptr, "null workspace");
  return bispec_plan_create(plan, d, b, est, ell, prec, ws, ws_bytes, as_stream(stream));
}

void cnpc_bispec_plan_destroy(cnpc_bispec_plan* plan) { bispec_plan_destroy(plan); }

int32_t cnpc_bispec_nconfigs(const cnpc_bispec_plan* p) { return p ? p->nconf : 0; }

cnpc_status cnpc_bispec_configs(const cnpc_bispec_plan* p, int32_t* ijk, int64_t* ntri) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr, "null plan");
  if (ijk) memcpy(ijk, p->cfg.data(), sizeof(int32_t) * 3 * p->nconf);
  if (ntri) memcpy(ntri, p->ntri.data(), sizeof(int64_t) * p->nconf);
  return CNPC_OK;
}

int32_t cnpc_bispec_band(const cnpc_bispec_plan* p) { return p ? p->band : 0; }

int32_t cnpc_bispec_grid(const cnpc_bispec_plan* p) { return p ? p->grid : 0; }

cnpc_status cnpc_bispec_ext_bins(const cnpc_bispec_plan* p, cnpc_kbins* ext) {
  API_BEGIN;
  CNPC_REQUIRE(p && ext, "null pointer argument");
  *ext = p->ext;
  return CNPC_OK;
}

cnpc_status cnpc_bispectrum(const cnpc_bispec_plan* p, const void* F0, const void* Fl,
                            const double* noise_means, const double* norms, double* raw, double* shot,
                            double* value, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr, "null plan");
  CNPC_REQUIRE(F0 && norms && raw && shot && value && ws, "null pointer argument");
  CNPC_REQUIRE(p->est == CNPC_EST_SCOCCIMARRO || p->est == CNPC_EST_TRIPOSH,
               "a Sugiyama plan runs through cnpc_sugiyama");
  CNPC_REQUIRE(p->ell == 0 || p->est == CNPC_EST_TRIPOSH || Fl != nullptr, "B_l with l > 0 needs F_l");
  CNPC_REQUIRE(p->est != CNPC_EST_TRIPOSH || Fl != nullptr, "TripoSH needs F_l (F_0 for l = 0)");
  return bispec_run(p, F0, Fl, nullptr, nullptr, noise_means, norms, raw, shot, value, ws, ws_bytes,
                    as_stream(stream));
}

size_t cnpc_bispec_indicator_bytes(const cnpc_bispec_plan* p) {
  if (p == nullptr || p->est != CNPC_EST_TRIPOSH) return 0;
  return bispec_indicator_bytes(p);
}

cnpc_status cnpc_bispec_indicators(const cnpc_bispec_plan* p, void* ind, void* ws, size_t ws_bytes,
                                   void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr, "null plan");
  CNPC_REQUIRE(p->est == CNPC_EST_TRIPOSH, "shell indicator fields serve the TripoSH FFT-method noise");
  CNPC_REQUIRE(ind && ws, "null pointer argument");
  return bispec_indicators(p, ind, ws, ws_bytes, as_stream(stream));
}

cnpc_status cnpc_bispectrum_fft_noise(const cnpc_bispec_plan* p, const void* F0, const void* Fl,
                                      const void* FN0, const void* ind, const double* noise_means,
                                      const double* norms, double* raw, double* shot, double* value, void* ws,
                                      size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr, "null plan");
  CNPC_REQUIRE(p->est == CNPC_EST_TRIPOSH, "the FFT-method shot noise is implemented for TripoSH plans");
  CNPC_REQUIRE(F0 && Fl && FN0 && ind && noise_means && norms && raw && shot && value && ws,
               "null pointer argument");
  return bispec_run(p, F0, Fl, FN0, ind, noise_means, norms, raw, shot, value, ws, ws_bytes,
                    as_stream(stream));
}

}  // extern "C"
