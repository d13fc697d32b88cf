// Host-side pieces of the bispectrum: plan, shell c2r, contraction, finalize.
#pragma once

#include <vector>

#include "spectra.h"

namespace cnpc {

constexpr int MAX_COLS = 40;

struct ContractCols {
  int ncols;
  int field[MAX_COLS];  // field index of each column
};

struct FinArgs {
  int est, ell, nb, next, ncols, nconf;
  double n3;
  const int* cfg;
  const int* prow;       // per config: its row of the contraction output
  const int64_t* ntri;
  const double* aux;     // per config: L(mu_ij), L(mu_ik) (Scoccimarro) or g(t), g(1/t)
  const double* counts;  // N_mode per shell
  const double* wq;      // N_c / k_c per extended bin
};

struct BispecGeom {
  int band;     // band half-width M of F_0 / F_l
  int grid;     // side G of the grid the shell fields and the contraction use
  int nfields;  // real fields per catalog
  int ncols;    // contraction columns
};

double g_ell_host(int l, double t);
BispecGeom bispec_geometry(const cnpc_mesh_desc* d, const cnpc_kbins* b, int est, int ell);
size_t bispec_ws_bytes(const cnpc_mesh_desc* d, const cnpc_kbins* b, int est, int ell);
// out[r][c] = sum_x X_a(x) X_b(x) Y_c(x) over the npts grid points, fields
// [nf][npts]: row r is the pair (a, b) = pairs[r] (a | b << 16, nlist rows)
// or, without a list, the r-th pair a <= b of the nshell first fields in
// (a, b) lexicographic order; column c is field cc.field[c].
template <typename T>
cnpc_status contract_valu(const T* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                          double* partial, double* out, hipStream_t s, const uint32_t* pairs = nullptr,
                          int nlist = 0);
cnpc_status contract_mfma(const float* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                          double* partial, double* out, hipStream_t s, const uint32_t* pairs = nullptr,
                          int nlist = 0);
// the same in the field type (FP32 or FP64) on the matrix cores
template <typename T>
cnpc_status contract_mfma_fp(const T* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                             double* partial, double* out, hipStream_t s, const uint32_t* pairs = nullptr,
                             int nlist = 0);

}  // namespace cnpc

struct cnpc_bispec_plan {
  cnpc_mesh_desc desc;
  cnpc_kbins bins, ext;
  int est, ell, prec;
  int nb, next, band, grid, nfields, nconf;
  cnpc::ContractCols cc;
  std::vector<int64_t> thr, counts, counts_ext, ntri;
  std::vector<int> cfg;
  std::vector<double> aux, wq;
  // contraction rows: the shell pairs the configurations use (a | b << 16), and
  // the row of each configuration
  std::vector<uint32_t> pairs;
  std::vector<int> prow;
  uint32_t* d_pairs = nullptr;
  int* d_prow = nullptr;
  int* d_cfg = nullptr;
  int64_t* d_ntri = nullptr;
  double* d_aux = nullptr;
  double* d_counts = nullptr;
  double* d_wq = nullptr;
  // Sugiyama B_l1l2L (estimator CNPC_EST_SUGIYAMA): multipoles, the paired
  // (m1, m2, M) sub-configurations with their weights eta (l1 l2 L; m1 m2 M),
  // H N, and the k3 weights of the i = j != k shot-noise term per (i, j)
  int l1 = 0, l2 = 0, L = 0;
  std::vector<int> sub;       // m1, m2, M, symmetry flag per sub-configuration
  std::vector<double> subw;   // weight per sub-configuration
  double hn = 0.0;            // (l1 l2 L; 0 0 0) (2l1+1)(2l2+1)(2L+1)
  double* d_wq3 = nullptr;    // [nb][nb][next]
};

namespace cnpc {
cnpc_status bispec_plan_create(cnpc_bispec_plan** out, const cnpc_mesh_desc* d, const cnpc_kbins* b,
                               int est, int ell, int prec, void* ws, size_t ws_bytes, hipStream_t s);
void bispec_plan_destroy(cnpc_bispec_plan* P);
cnpc_status bispec_run(const cnpc_bispec_plan* P, const void* F0, const void* Fl, const void* FN0,
                       const void* ind, const double* noise, const double* norms, double* raw, double* shot,
                       double* value, void* ws, size_t ws_bytes, hipStream_t s);
size_t bispec_indicator_bytes(const cnpc_bispec_plan* P);
cnpc_status bispec_indicators(const cnpc_bispec_plan* P, void* out, void* ws, size_t ws_bytes, hipStream_t s);
}  // namespace cnpc
