// Host-side entry points of the catalog sums and the painter.
#pragma once

#include "common.h"

namespace cnpc {

struct SumsArgs {
  int lmax;  // Y_lm sums for l <= lmax (0, 2 or 4); the others stay zero
  double boxsize;
  double obs[3];
  double los[3];
  int global_los;
};

template <typename T>
struct FoldArgs {
  const T* blocks[4];
  int n, nt, nphase, nsets;
};

struct PaintLayout {
  int nt, ntiles, nphase, nsets, nbuckets;
  size_t off_rec, off_tmp;  // sorted records, bucket-ordered records (shared by both catalogs)
  size_t off_count[2];           // tile counts of the galaxy / random catalog
  size_t off_partial, off_sums;  // catalog-sum partials and sums (fused entry point)
  size_t off_start, off_cursor, off_bcur;
  size_t off_blocks[4];
  // fused bucket pass (entry point with catalog sums, more than one bucket):
  // fixed-capacity bucket regions, the overflow records, the bucket
  // reservation counters (+ one overflow counter)
  uint32_t cap;
  size_t off_region, off_ovf, off_bcnt;
  size_t total;
};

PaintLayout paint_layout(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, bool weighted);
cnpc_status launch_catalog_sums(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w,
                                int64_t n, double* sums, void* ws, size_t ws_bytes, hipStream_t s);
cnpc_status launch_norms(const cnpc_mesh_desc* d, const double* gs, const double* rs, int64_t ngal,
                         double* norms, hipStream_t s);
cnpc_status launch_paint(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                         int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                         const double* norms, void* delta, void* noise, void* ws, size_t ws_bytes,
                         hipStream_t s);
cnpc_status launch_paint_fkp(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                             int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                             int sums_lmax, double* gsums, double* rsums, double* norms, void* delta,
                             void* noise, void* ws, size_t ws_bytes, hipStream_t s);
// Painting into tile blocks (sums, sort, tile painting; no fold), then the
// fold fused with the r2c z pass of both de-interlacing transforms: dsp gets
// the delta z rows [phase][x][y][n/2] (complex), nw1 the N z rows
// [phase][x][y][m].  Interlaced meshes of side 256 with the register FFT
// passes (has_fold_zr2c); the blocks live in ws up to paint_layout().total.
bool has_fold_zr2c(const cnpc_mesh_desc* d);
cnpc_status launch_paint_blocks_zr2c(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw, int64_t ngal,
                                     const uint32_t* rpos, const float* rw, int64_t nran, int sums_lmax,
                                     double* gsums, double* rsums, double* norms, void* dsp, void* nw1, int m,
                                     void* ws, size_t ws_bytes, hipStream_t s);
// per-workgroup LDS limit of the current device (bytes)
size_t lds_limit();

}  // namespace cnpc
