// Host-side entry points of the Y_lm transforms, de-interlacing, F_l assembly
// and binning kernels.
#pragma once

#include <algorithm>

#include "fft.h"
#include "paint.h"

namespace cnpc {

constexpr int MAX_PAIRS = 16;
constexpr int MAX_SELF = 4;

template <typename T>
struct BinArgs {
  int n, m, assign, interlace, nbins, npairs, nself;
  int self_ell[MAX_SELF];
  int64_t thr[MAX_BINS + 1];
  const cx<T>* pa[MAX_PAIRS];
  const cx<T>* pb[MAX_PAIRS];
  uint32_t imag;  // bit q: pair q accumulates Im F_a F_b^* instead of Re
};

template <typename T>
cnpc_status band_forward_yx(int n, int dt, int batch, int m, const cx<T>* w1, cx<T>* w2, cx<T>* out,
                            hipStream_t s);
size_t ylm_r2c_ws_bytes(const cnpc_mesh_desc* d, int nfields, int band);
// coef: the table of launch_ylm_coef for the same mesh, ells and band, or
// nullptr (the call forms it in its workspace).  delta_zspec: delta holds the
// z half spectra that launch_paint_deinterlace leaves with delta_int_zspec
// (the real mesh is then never stored); only where ylm_coef_bytes > 0.
cnpc_status launch_ylm_r2c(const cnpc_mesh_desc* d, int band, int nells, const int32_t* ells,
                           const void* delta, void* out, void* ws, size_t ws_bytes, hipStream_t s,
                           const void* coef = nullptr, bool delta_zspec = false);
// Per-row coefficient table of the FP32 z-power-bases route of launch_ylm_r2c:
// its bytes (0 when that route does not apply) and a kernel that fills it.
size_t ylm_coef_bytes(const cnpc_mesh_desc* d, int nells, const int32_t* ells, int band);
cnpc_status launch_ylm_coef(const cnpc_mesh_desc* d, int nells, const int32_t* ells, int band, void* coef,
                            hipStream_t s);
cnpc_status launch_ylm_fields(const cnpc_mesh_desc* d, int ell, const void* delta, void* out,
                              hipStream_t s);
size_t deinterlace_ws_bytes(const cnpc_mesh_desc* d);
size_t deinterlace_ws_max(const cnpc_mesh_desc* d);
// Painting (sums, sort, tile painting) with the fold fused into the z passes
// of the de-interlacing transforms (has_fold_zr2c meshes): the same outputs as
// launch_paint_fkp followed by launch_deinterlace of delta (full, with
// delta_int) and of N (band), without the delta and N meshes.
size_t paint_deinterlace_ws_bytes(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, bool weighted, int band);
cnpc_status launch_paint_deinterlace(const cnpc_mesh_desc* d, int band, const uint32_t* gpos, const float* gw,
                                     int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                                     int sums_lmax, double* gsums, double* rsums, double* norms, void* spec,
                                     void* delta_int, void* specN, void* ws, size_t ws_bytes, hipStream_t s,
                                     bool delta_int_zspec = false);
size_t deinterlace_band_ws_bytes(const cnpc_mesh_desc* d, int band);
cnpc_status launch_deinterlace(const cnpc_mesh_desc* d, int band, const void* meshes, void* spec,
                               void* delta_int, void* ws, size_t ws_bytes, hipStream_t s);
cnpc_status launch_assemble(const cnpc_mesh_desc* d, int band, int ell, const void* spec0,
                            const void* ylm, void* F, hipStream_t s);
size_t bin_ws_doubles(int nbins, int npairs, int nself);
cnpc_status launch_bin(const cnpc_mesh_desc* d, const int64_t* thr, int nbins, int band, int npairs,
                       const void* const* pa, const void* const* pb, uint32_t imag, int nself,
                       const int32_t* self_ells, const double* norms, double* acc, double* means,
                       double* selfterm, int64_t* nmodes, double* keff, hipStream_t s);
cnpc_status launch_pk_multipole(int nbins, int ell, const double* mean, const double* norms, double* out,
                                hipStream_t s);
cnpc_status launch_cross_norms(const double* na, const double* nb, double* out, hipStream_t s);
cnpc_status launch_pk_finalize(int nbins, const double* m00, const double* m02, const double* m04,
                               const double* m22, const double* m42, const double* m44,
                               const double* norms, double* out, hipStream_t s);

}  // namespace cnpc
