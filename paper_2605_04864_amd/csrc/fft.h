// Host-side entry points of the FFT building blocks.
#pragma once

#include "fft_device.h"

namespace cnpc {

constexpr int MAX_BINS = 128;

struct ColArgs {
  int64_t plane_in, plane_out;  // element strides between planes
  int64_t row_in, row_out;      // element strides between rows (transform index)
  int ncols;                    // contiguous columns per plane (multiple of W)
  int W, logW;                  // column tile width
  int band_in, band_out;        // 0: all N rows stored; M: only the 2M band rows
  // optional shell mask on input (x pass of a band c2r): plane p keeps the
  // modes with thr[mask_b0 + p] <= |n|^2 < thr[mask_b0 + p + 1]; columns are
  // (jy, kz) of a band layout of half-width mask_m.  mask_m == 0: no mask.
  int mask_m, mask_b0;
  int64_t thr[MAX_BINS + 1];
};

cnpc_status ensure_twiddles();
size_t lds_limit();
int col_tile_width(int n, int dtype);
ColArgs make_col(int n, int dtype, int64_t plane_in, int64_t plane_out, int64_t row_in,
                 int64_t row_out, int ncols, int band_in, int band_out);

template <typename T>
cnpc_status zpass_r2c(int n, const T* in, cx<T>* out, int64_t nrows, int kz, hipStream_t s);
template <typename T>
cnpc_status zpass_c2r(int n, const cx<T>* in, T* out, int64_t nrows, int kz, hipStream_t s);
template <typename T>
cnpc_status colpass(int n, int dir, const cx<T>* in, cx<T>* out, const ColArgs& a, int64_t nplanes,
                    hipStream_t s);
template <typename T>
cnpc_status fft3d_r2c(int n, int batch, int band, const T* in, cx<T>* out, cx<T>* ws, hipStream_t s);
template <typename T>
cnpc_status fft3d_c2r(int n, int batch, int band, const cx<T>* in, T* out, cx<T>* ws, hipStream_t s);
// fused x pass of the interlaced full transform (N = 64 or 256; see fft.hip)
template <typename T>
cnpc_status xpass_interlace(int n, const cx<T>* in, cx<T>* out, cx<T>* band_out, int mb, T scale,
                            hipStream_t s);
inline bool has_xpass_interlace(int n) { return (n == 64 || n == 256) && fft_register_passes(); }
// complex elements of scratch needed by fft3d_* (0 for full transforms)
size_t fft_ws_elems(int n, int batch, int band);

}  // namespace cnpc
