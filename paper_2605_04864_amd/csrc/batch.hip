// Native batched runner of the combined power-spectrum / bispectrum workload:
// every catalog pair through paint -> de-interlace -> Y_lm transforms -> F_l
// assembly -> shell means -> P_l -> Scoccimarro B_0, catalogs spread
// round-robin over streams owned by the batch, each stream with its own slab
// of the caller's workspace; optionally captured once into a HIP graph and
// replayed.
#include "bispec.h"

namespace cnpc {

constexpr int BATCH_MAX_STREAMS = 16;
constexpr int BATCH_MAX_ELLS = 3;

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace cnpc

struct cnpc_batch {
  cnpc_mesh_desc desc;
  cnpc_kbins bins;
  const cnpc_bispec_plan* plan;
  int nells = 0, ells[cnpc::BATCH_MAX_ELLS] = {0, 0, 0};
  int nhi = 0, his[cnpc::BATCH_MAX_ELLS] = {0, 0, 0}, nf = 0;
  int nstreams = 0, band = 0, sums_lmax = 0;
  int64_t max_ngal = 0, max_nran = 0;
  int64_t thr[cnpc::MAX_BINS + 1];
  // slab layout (bytes from the slab start)
  size_t o_norms, o_gs, o_rs, o_delta, o_noise, o_D, o_DN, o_dint, o_ylm, o_F[cnpc::BATCH_MAX_ELLS], o_FN0,
      o_means, o_nmodes, o_keff, o_call, call_bytes, slab;
  size_t shared = 0;  // bytes before the slabs: the Y_lm coefficient table shared by every catalog
  std::vector<hipStream_t> streams;
  hipStream_t origin = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace cnpc {

static void batch_free(cnpc_batch* B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (hipEvent_t e : B->join)
    if (e) (void)hipEventDestroy(e);
  if (B->fork) (void)hipEventDestroy(B->fork);
  for (hipStream_t s : B->streams)
    if (s) (void)hipStreamDestroy(s);
  if (B->origin) (void)hipStreamDestroy(B->origin);
  delete B;
}

static void batch_layout(cnpc_batch* B) {
  const cnpc_mesh_desc* d = &B->desc;
  const size_t es = esize(d->dtype);
  const size_t n3 = (size_t)d->n * d->n * d->n;
  const size_t nph = d->interlace ? 2 : 1;
  const size_t bsz = (size_t)4 * B->band * B->band * B->band * 2 * es;  // one band spectrum
  const int nb = B->bins.nbins;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = al256(o + bytes); return at; };
  B->o_norms = take(sizeof(double) * CNPC_NORMS_LEN);
  B->o_gs = take(sizeof(double) * CNPC_SUMS_LEN);
  B->o_rs = take(sizeof(double) * CNPC_SUMS_LEN);
  B->o_delta = take(nph * n3 * es);
  B->o_noise = take(nph * n3 * es);
  B->o_D = take(bsz);
  B->o_DN = take(bsz);
  B->o_dint = B->nhi ? take(n3 * es) : 0;
  B->o_ylm = B->nhi ? take((size_t)B->nf * bsz) : 0;
  for (int q = 0; q < B->nells; ++q) B->o_F[q] = take(bsz);
  B->o_FN0 = take(bsz);
  // shell means: the pairs (F_0, F_l) of the ells, then (F_0, N_0) twice and
  // the self term, so that the last three rows are the Q, H, s rows of the
  // B_0 shot noise
  B->o_means = take(sizeof(double) * (size_t)(B->nells + 3) * nb);
  B->o_nmodes = take(sizeof(int64_t) * nb);
  B->o_keff = take(sizeof(double) * nb);
  size_t call = paint_layout(d, B->max_ngal, B->max_nran, true).total;
  if (has_fold_zr2c(d) && B->nhi)
    call = std::max(call, paint_deinterlace_ws_bytes(d, B->max_ngal, B->max_nran, true, B->band));
  call = std::max(call, deinterlace_ws_max(d));
  if (B->nhi) call = std::max(call, ylm_r2c_ws_bytes(d, B->nf, B->band));
  call = std::max(call, bin_ws_doubles(nb, B->nells + 1, 1) * sizeof(double));
  call = std::max(call, bispec_ws_bytes(d, &B->bins, CNPC_EST_SCOCCIMARRO, 0));
  B->call_bytes = call;
  B->o_call = take(call);
  B->slab = o;
  B->shared = B->nhi ? al256(ylm_coef_bytes(d, B->nhi, B->his, B->band)) : 0;
}

struct BatchArgs {
  int ncat;
  const uint32_t* const* gpos;
  const float* const* gw;
  const int64_t* ngal;
  const uint32_t* const* rpos;
  const float* const* rw;
  const int64_t* nran;
  double* const* pk;
  double* const* bk;
  unsigned char* ws;
};

static cnpc_status batch_catalog(const cnpc_batch* B, const BatchArgs& a, int i, unsigned char* w,
                                 const void* coef, hipStream_t s) {
  const cnpc_mesh_desc* d = &B->desc;
  const int nb = B->bins.nbins, band = B->band, nl = B->nells;
  double* norms = reinterpret_cast<double*>(w + B->o_norms);
  void* delta = w + B->o_delta;
  void* noise = w + B->o_noise;
  void* D = w + B->o_D;
  void* DN = w + B->o_DN;
  void* dint = B->nhi ? w + B->o_dint : nullptr;
  void* call = w + B->o_call;
  const size_t bsz = (size_t)4 * band * band * band * 2 * esize(d->dtype);
  const float* gw = a.gw ? a.gw[i] : nullptr;
  const float* rw = a.rw ? a.rw[i] : nullptr;
  double* gs = reinterpret_cast<double*>(w + B->o_gs);
  double* rs = reinterpret_cast<double*>(w + B->o_rs);
  // FP32 z-power-bases route of the Y_lm transforms: the de-aliased mesh stays
  // as z half spectra and its inverse z pass runs inside the Y_lm z pass
  bool zspec = false;
  if (dint && has_fold_zr2c(d) && tune_value(CNPC_TUNE_FOLD_FUSED) != 1) {
    // fold fused with the z passes of both de-interlacing transforms
    zspec = B->nhi && ylm_coef_bytes(d, B->nhi, B->his, band) > 0;
    CNPC_TRY(launch_paint_deinterlace(d, band, a.gpos[i], gw, a.ngal[i], a.rpos[i], rw, a.nran[i], B->sums_lmax, gs,
                                      rs, norms, D, dint, DN, call, B->call_bytes, s, zspec));
  } else {
    CNPC_TRY(launch_paint_fkp(d, a.gpos[i], gw, a.ngal[i], a.rpos[i], rw, a.nran[i], B->sums_lmax, gs, rs, norms,
                              delta, noise, call, B->call_bytes, s));
    CNPC_TRY(launch_deinterlace(d, band, delta, D, dint, call, B->call_bytes, s));
    CNPC_TRY(launch_deinterlace(d, band, noise, DN, nullptr, call, B->call_bytes, s));
  }
  void* F[BATCH_MAX_ELLS] = {nullptr, nullptr, nullptr};
  for (int q = 0; q < nl; ++q) F[q] = w + B->o_F[q];
  void* FN0 = w + B->o_FN0;
  void* F0 = nullptr;
  for (int q = 0; q < nl; ++q)
    if (B->ells[q] == 0) F0 = F[q];
  CNPC_TRY(launch_assemble(d, band, 0, D, nullptr, F0, s));
  CNPC_TRY(launch_assemble(d, band, 0, DN, nullptr, FN0, s));
  if (B->nhi) {
    unsigned char* ylm = w + B->o_ylm;
    CNPC_TRY(launch_ylm_r2c(d, band, B->nhi, B->his, dint, ylm, call, B->call_bytes, s, coef, zspec));
    size_t f = 0;
    for (int h = 0; h < B->nhi; ++h) {
      const int l = B->his[h];
      for (int q = 0; q < nl; ++q)
        if (B->ells[q] == l) CNPC_TRY(launch_assemble(d, band, l, nullptr, ylm + f * bsz, F[q], s));
      f += 2 * l + 1;
    }
  }
  const void* pa[BATCH_MAX_ELLS + 1];
  const void* pb[BATCH_MAX_ELLS + 1];
  for (int q = 0; q < nl; ++q) { pa[q] = F0; pb[q] = F[q]; }
  pa[nl] = F0;
  pb[nl] = FN0;
  double* means = reinterpret_cast<double*>(w + B->o_means);
  const int32_t self0[1] = {0};
  CNPC_TRY(launch_bin(d, B->thr, nb, band, nl + 1, pa, pb, 0u, 1, self0, norms, reinterpret_cast<double*>(call),
                      means, means + (size_t)(nl + 2) * nb, reinterpret_cast<int64_t*>(w + B->o_nmodes),
                      reinterpret_cast<double*>(w + B->o_keff), s));
  hipLaunchKernelGGL(k_copy_f64, dim3((nb + 63) / 64), dim3(64), 0, s, means + (size_t)nl * nb,
                     means + (size_t)(nl + 1) * nb, nb);
  CNPC_HIP(hipGetLastError());
  const double* m[3] = {nullptr, nullptr, nullptr};  // l = 0, 2, 4
  for (int q = 0; q < nl; ++q) m[B->ells[q] / 2] = means + (size_t)q * nb;
  CNPC_TRY(launch_pk_finalize(nb, m[0], m[1], m[2], nullptr, nullptr, nullptr, norms, a.pk[i], s));
  const int nc = B->plan->nconf;
  double* bk = a.bk[i];
  return bispec_run(B->plan, F0, nullptr, nullptr, nullptr, means + (size_t)nl * nb, norms, bk, bk + nc,
                    bk + 2 * (size_t)nc, call, B->call_bytes, s);
}

// form the shared tables on s0, fork the batch streams from s0, enqueue every
// catalog, join them back into s0
static cnpc_status batch_enqueue(const cnpc_batch* B, const BatchArgs& a, hipStream_t s0) {
  const void* coef = nullptr;
  const size_t cb = B->shared ? ylm_coef_bytes(&B->desc, B->nhi, B->his, B->band) : 0;  // 0: another route now
  if (cb > 0 && cb <= B->shared) {
    CNPC_TRY(launch_ylm_coef(&B->desc, B->nhi, B->his, B->band, a.ws, s0));
    coef = a.ws;
  }
  CNPC_HIP(hipEventRecord(B->fork, s0));
  for (hipStream_t s : B->streams) CNPC_HIP(hipStreamWaitEvent(s, B->fork, 0));
  cnpc_status st = CNPC_OK;
  for (int i = 0; i < a.ncat && st == CNPC_OK; ++i) {
    const int k = i % B->nstreams;
    st = batch_catalog(B, a, i, a.ws + B->shared + (size_t)k * B->slab, coef, B->streams[k]);
  }
  // join even after a failed enqueue, so that a capture can end cleanly
  for (int k = 0; k < B->nstreams; ++k) {
    CNPC_HIP(hipEventRecord(B->join[k], B->streams[k]));
    CNPC_HIP(hipStreamWaitEvent(s0, B->join[k], 0));
  }
  return st;
}

}  // namespace cnpc

using namespace cnpc;

static cnpc_status batch_check_args(const cnpc_batch* B, const BatchArgs& a, size_t ws_bytes) {
  CNPC_REQUIRE(a.ncat >= 1, "need at least one catalog");
  CNPC_REQUIRE(a.gpos && a.ngal && a.rpos && a.nran && a.pk && a.bk && a.ws, "null pointer argument");
  CNPC_REQUIRE((a.gw == nullptr) == (a.rw == nullptr), "give weight arrays for both catalogs or for neither");
  if (ws_bytes < B->shared + (size_t)B->nstreams * B->slab) {
    set_error("batch workspace too small: need %zu, got %zu", B->shared + (size_t)B->nstreams * B->slab, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  for (int i = 0; i < a.ncat; ++i) {
    CNPC_REQUIRE(a.gpos[i] && a.rpos[i] && a.pk[i] && a.bk[i], "null pointer for catalog %d", i);
    CNPC_REQUIRE(a.ngal[i] >= 1 && a.ngal[i] <= B->max_ngal, "catalog %d: ngal %lld outside [1, %lld]", i,
                 (long long)a.ngal[i], (long long)B->max_ngal);
    CNPC_REQUIRE(a.nran[i] >= 1 && a.nran[i] <= B->max_nran, "catalog %d: nran %lld outside [1, %lld]", i,
                 (long long)a.nran[i], (long long)B->max_nran);
    if (a.gw) CNPC_REQUIRE((a.gw[i] == nullptr) == (a.rw[i] == nullptr), "catalog %d: weights for one side only", i);
  }
  return CNPC_OK;
}

extern "C" {

cnpc_status cnpc_batch_create(cnpc_batch** out, const cnpc_mesh_desc* d, const cnpc_kbins* b,
                              const cnpc_bispec_plan* plan, int32_t nells, const int32_t* ells,
                              int32_t nstreams, int64_t max_ngal, int64_t max_nran) {
  API_BEGIN;
  CNPC_REQUIRE(out != nullptr, "null batch pointer");
  *out = nullptr;
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_bins(d, b));
  CNPC_REQUIRE(plan != nullptr, "null plan");
  CNPC_REQUIRE(plan->est == CNPC_EST_SCOCCIMARRO && plan->ell == 0, "the batch measures the Scoccimarro B_0");
  CNPC_REQUIRE(plan->desc.n == d->n && plan->desc.dtype == d->dtype && plan->desc.assign == d->assign &&
                   plan->desc.interlace == d->interlace && plan->desc.boxsize == d->boxsize,
               "the plan was made for another mesh");
  CNPC_REQUIRE(plan->bins.kmin == b->kmin && plan->bins.dk == b->dk && plan->bins.nbins == b->nbins,
               "the plan was made for other bins");
  CNPC_REQUIRE(nells >= 1 && nells <= BATCH_MAX_ELLS && ells != nullptr, "need 1 to %d multipoles",
               BATCH_MAX_ELLS);
  bool has0 = false;
  for (int q = 0; q < nells; ++q) {
    CNPC_REQUIRE(ells[q] == 0 || ells[q] == 2 || ells[q] == 4, "ells must be 0, 2 or 4");
    for (int p = 0; p < q; ++p) CNPC_REQUIRE(ells[p] != ells[q], "repeated multipole %d", ells[q]);
    has0 = has0 || ells[q] == 0;
  }
  CNPC_REQUIRE(has0, "the multipoles must include l = 0");
  CNPC_REQUIRE(nstreams >= 1 && nstreams <= BATCH_MAX_STREAMS, "nstreams must be in [1, %d]", BATCH_MAX_STREAMS);
  CNPC_REQUIRE(max_ngal >= 1 && max_ngal < ((int64_t)1 << 32), "max_ngal must be in [1, 2^32)");
  CNPC_REQUIRE(max_nran >= 1 && max_nran < ((int64_t)1 << 32), "max_nran must be in [1, 2^32)");
  auto* B = new cnpc_batch();
  B->desc = *d;
  B->bins = *b;
  B->plan = plan;
  B->nells = nells;
  for (int q = 0; q < nells; ++q) {
    B->ells[q] = ells[q];
    if (ells[q] > 0) {
      B->his[B->nhi++] = ells[q];
      B->nf += 2 * ells[q] + 1;
    }
  }
  B->nstreams = nstreams;
  B->band = plan->band;
  B->sums_lmax = 0;  // P_l and the B_0 shot noise need the l = 0 catalog sums only
  B->max_ngal = max_ngal;
  B->max_nran = max_nran;
  bin_thresholds(d, b, B->thr);
  batch_layout(B);
  // one-time device set-up before any capture
  cnpc_status st = ensure_twiddles();
  (void)lds_limit();
  for (int k = 0; st == CNPC_OK && k < nstreams; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      set_error("hipStreamCreateWithFlags failed");
      st = CNPC_EHIP;
      break;
    }
    B->streams.push_back(s);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      set_error("hipEventCreateWithFlags failed");
      st = CNPC_EHIP;
      break;
    }
    B->join.push_back(e);
  }
  if (st == CNPC_OK && (hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess)) {
    set_error("stream or event creation failed");
    st = CNPC_EHIP;
  }
  if (st != CNPC_OK) {
    batch_free(B);
    return st;
  }
  *out = B;
  return CNPC_OK;
}

size_t cnpc_batch_workspace_size(const cnpc_batch* B) { return B ? B->shared + (size_t)B->nstreams * B->slab : 0; }

void cnpc_batch_destroy(cnpc_batch* B) { batch_free(B); }

cnpc_status cnpc_batch_run(cnpc_batch* B, int32_t ncat, const uint32_t* const* gpos, const float* const* gw,
                           const int64_t* ngal, const uint32_t* const* rpos, const float* const* rw,
                           const int64_t* nran, double* const* pk_out, double* const* bk_out, void* ws,
                           size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(B != nullptr, "null batch");
  const BatchArgs a{ncat, gpos, gw, ngal, rpos, rw, nran, pk_out, bk_out, static_cast<unsigned char*>(ws)};
  CNPC_TRY(batch_check_args(B, a, ws_bytes));
  return batch_enqueue(B, a, as_stream(stream));
}

cnpc_status cnpc_batch_capture(cnpc_batch* B, int32_t ncat, const uint32_t* const* gpos, const float* const* gw,
                               const int64_t* ngal, const uint32_t* const* rpos, const float* const* rw,
                               const int64_t* nran, double* const* pk_out, double* const* bk_out, void* ws,
                               size_t ws_bytes) {
  API_BEGIN;
  CNPC_REQUIRE(B != nullptr, "null batch");
  const BatchArgs a{ncat, gpos, gw, ngal, rpos, rw, nran, pk_out, bk_out, static_cast<unsigned char*>(ws)};
  CNPC_TRY(batch_check_args(B, a, ws_bytes));
  if (B->exec) { (void)hipGraphExecDestroy(B->exec); B->exec = nullptr; }
  if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
  CNPC_HIP(hipStreamBeginCapture(B->origin, hipStreamCaptureModeThreadLocal));
  const cnpc_status st = batch_enqueue(B, a, B->origin);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(B->origin, &g);
  if (st != CNPC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ec != hipSuccess || g == nullptr) {
    set_error("graph capture failed: %s", hipGetErrorString(ec));
    return CNPC_EHIP;
  }
  B->graph = g;
  CNPC_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  return CNPC_OK;
}

cnpc_status cnpc_batch_replay(cnpc_batch* B, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(B != nullptr, "null batch");
  CNPC_REQUIRE(B->exec != nullptr, "nothing captured: call cnpc_batch_capture first");
  CNPC_HIP(hipGraphLaunch(B->exec, as_stream(stream)));
  return CNPC_OK;
}

}  // extern "C"
