// Batched 3-D real FFTs for gfx950: z-row passes (two real rows packed in one
// complex transform), strided column passes (x and y), band pruning.
#include <mutex>
#include <type_traits>
#include <vector>
#include <cmath>

#include "fft.h"

namespace cnpc {

__device__ cx<double> g_twiddle1024[1024];

cnpc_status ensure_twiddles() {
  static std::mutex mu;
  static bool ready[64] = {false};
  int dev = 0;
  CNPC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index %d out of range", dev);
    return CNPC_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (ready[dev]) return CNPC_OK;
  std::vector<cx<double>> h(1024);
  for (int t = 0; t < 1024; ++t) {
    // exp(-2 pi i t / 1024) via exact octant symmetry of the angle
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * t / 1024.0L;
    h[t] = cx<double>{(double)cosl(a), (double)(-sinl(a))};
  }
  CNPC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle1024), h.data(), sizeof(cx<double>) * 1024));
  ready[dev] = true;
  return CNPC_OK;
}

// ------------------------------------------------------------------ sizes --
template <typename T, int N>
struct ZCfg {
  // sequences per workgroup so that the two ping-pong buffers take <= 32 KiB
  static constexpr int bytes = 16384;
  static constexpr int nseq_raw = bytes / (N * (int)sizeof(cx<T>));
  static constexpr int NSEQ = nseq_raw < 1 ? 1 : nseq_raw;
};

int col_tile_width(int n, int dtype) {
  // 128-byte row segments (or the tuned width) when LDS allows: twiddles +
  // two buffers of N x W elements
  const size_t es = dtype == CNPC_F64 ? 16 : 8;
  const size_t lim = lds_limit();
  const int tw = tune_value(CNPC_TUNE_FFT_COL_W);
  int w = tw > 0 ? tw : (int)(128 / es);
  while (w > 1 && (2 * (size_t)n * w + n) * es > lim) w >>= 1;
  return w;
}

// ---------------------------------------------------------- z-pass r2c --
// rows r = 0..nrows-1 of length N (real, in + r*N); pairs (2q, 2q+1) packed as
// one complex sequence z = a + i b.  Output row r: kz = 0..kz_keep-1 complex at
// out + r * kz_keep.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_zpass_r2c(const T* __restrict__ in, cx<T>* __restrict__ out,
                                                   int64_t npairs, int kz_keep) {
  constexpr int NSEQ = ZCfg<T, N>::NSEQ;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* A = tw + N;
  cx<T>* B = A + NSEQ * N;
  load_twiddles<T, N, -1>(tw);
  const int64_t q0 = (int64_t)blockIdx.x * NSEQ;
  const int nq = (int)((npairs - q0) < NSEQ ? (npairs - q0) : NSEQ);
  for (int idx = threadIdx.x; idx < nq * N; idx += blockDim.x) {
    const int s = idx / N, e = idx - s * N;
    const T* r0 = in + (2 * (q0 + s)) * (int64_t)N;
    A[s * N + e] = cx<T>{r0[e], r0[N + e]};
  }
  __syncthreads();
  cx<T>* Z = fft_lds<T, N, -1, false>(A, B, nq, 0, N, 1, tw);
  for (int idx = threadIdx.x; idx < nq * kz_keep; idx += blockDim.x) {
    const int s = idx / kz_keep, k = idx - s * kz_keep;
    const cx<T> zk = Z[s * N + k];
    const cx<T> zm = cconj(Z[s * N + ((N - k) & (N - 1))]);
    const cx<T> a = cscale(cadd(zk, zm), T(0.5));
    const cx<T> d = csub(zk, zm);
    const cx<T> b = {T(0.5) * d.y, T(-0.5) * d.x};  // (zk - zm) / (2 i)
    cx<T>* o = out + (2 * (q0 + s)) * (int64_t)kz_keep;
    o[k] = a;
    o[kz_keep + k] = b;
  }
}

// ---------------------------------------------------------- z-pass c2r --
// input rows r: kz = 0..kz_in-1 complex at in + r * kz_in (higher kz, and
// kz = N/2, taken as zero); output real rows at out + r * N.  in and out may
// alias when kz_in == N/2 (the workgroup reads all its rows first).
template <typename T, int N>
__global__ void __launch_bounds__(256) k_zpass_c2r(const cx<T>* in, T* out, int64_t npairs,
                                                   int kz_in) {
  constexpr int NSEQ = ZCfg<T, N>::NSEQ;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* A = tw + N;
  cx<T>* B = A + NSEQ * N;
  load_twiddles<T, N, 1>(tw);
  const int64_t q0 = (int64_t)blockIdx.x * NSEQ;
  const int nq = (int)((npairs - q0) < NSEQ ? (npairs - q0) : NSEQ);
  for (int idx = threadIdx.x; idx < nq * N; idx += blockDim.x) {
    const int s = idx / N, k = idx - s * N;
    const cx<T>* r0 = in + (2 * (q0 + s)) * (int64_t)kz_in;
    cx<T> z = {T(0), T(0)};
    if (k < (N >> 1)) {
      if (k < kz_in) {
        const cx<T> a = r0[k], b = r0[kz_in + k];
        z = cx<T>{a.x - b.y, a.y + b.x};
      }
    } else if (k > (N >> 1)) {
      const int kk = N - k;
      if (kk < kz_in) {
        const cx<T> a = r0[kk], b = r0[kz_in + kk];
        z = cx<T>{a.x + b.y, b.x - a.y};
      }
    }
    A[s * N + k] = z;
  }
  __syncthreads();
  cx<T>* Z = fft_lds<T, N, 1, false>(A, B, nq, 0, N, 1, tw);
  for (int idx = threadIdx.x; idx < nq * N; idx += blockDim.x) {
    const int s = idx / N, e = idx - s * N;
    T* o = out + (2 * (q0 + s)) * (int64_t)N;
    const cx<T> z = Z[s * N + e];
    o[e] = z.x;
    o[N + e] = z.y;
  }
}

// ------------------------------------------------- register z-passes --
// N = R^2: a group of R lanes transforms one row pair with row_fft_rr
// (256 / R row pairs per workgroup); same layouts and semantics as
// k_zpass_r2c / k_zpass_c2r.
template <typename T, int R>
__global__ void __launch_bounds__(256) k_zpass_r2c_rr(const T* __restrict__ in, cx<T>* __restrict__ out,
                                                      int64_t npairs, int kz_keep) {
  constexpr int N = R * R, GR = 256 / R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T, N, -1>(tw);
  const int grp = threadIdx.x / R, rank = threadIdx.x % R;
  cx<T>* buf = tw + N + grp * (R * (R + 1));
  const int64_t q = (int64_t)blockIdx.x * GR + grp;
  const bool live = q < npairs;
  const T* r0 = in + 2 * q * (int64_t)N;
  cx<T> v[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int z = rank + R * n2;
    v[n2] = live ? cx<T>{r0[z], r0[N + z]} : cx<T>{T(0), T(0)};
  }
  __syncthreads();
  row_fft_rr<T, R, -1>(v, rank, buf, tw);
  const int src = (R - rank) & (R - 1);
  const int K2 = (kz_keep + R - 1) / R;
  cx<T>* o = out + 2 * q * (int64_t)kz_keep;
#pragma unroll
  for (int k2 = 0; k2 < R / 2; ++k2) {
    if (k2 < K2) {
      const cx<T> a = v[R - 1 - k2];
      const cx<T> sh = {__shfl(a.x, src, R), __shfl(a.y, src, R)};
      const cx<T> zm = cconj(rank ? sh : v[(R - k2) & (R - 1)]);
      const cx<T> zk = v[k2];
      const int k = rank + R * k2;
      if (live && k < kz_keep) {
        const cx<T> dd = csub(zk, zm);
        o[k] = cscale(cadd(zk, zm), T(0.5));
        o[kz_keep + k] = cx<T>{T(0.5) * dd.y, T(-0.5) * dd.x};
      }
    }
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_zpass_c2r_rr(const cx<T>* in, T* out, int64_t npairs, int kz_in) {
  constexpr int N = R * R, GR = 256 / R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T, N, 1>(tw);
  const int grp = threadIdx.x / R, rank = threadIdx.x % R;
  cx<T>* buf = tw + N + grp * (R * (R + 1));
  const int64_t q = (int64_t)blockIdx.x * GR + grp;
  const bool live = q < npairs;
  const cx<T>* r0 = in + 2 * q * (int64_t)kz_in;
  cx<T> v[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int k = rank + R * n2;
    cx<T> z = {T(0), T(0)};
    if (live) {
      if (k < (N >> 1)) {
        if (k < kz_in) {
          const cx<T> a = r0[k], b = r0[kz_in + k];
          z = cx<T>{a.x - b.y, a.y + b.x};
        }
      } else if (k > (N >> 1)) {
        const int kk = N - k;
        if (kk < kz_in) {
          const cx<T> a = r0[kk], b = r0[kz_in + kk];
          z = cx<T>{a.x + b.y, b.x - a.y};
        }
      }
    }
    v[n2] = z;
  }
  __syncthreads();
  row_fft_rr<T, R, 1>(v, rank, buf, tw);
  if (live) {
    T* o = out + 2 * q * (int64_t)N;
#pragma unroll
    for (int k2 = 0; k2 < R; ++k2) {
      const int e = rank + R * k2;
      o[e] = v[k2].x;
      o[N + e] = v[k2].y;
    }
  }
}

// ---------------------------------------------------------- column pass --
// For each plane p and each tile of W consecutive columns: transform along the
// row index (length N).  Input rows: all N (band_in == 0) or the 2*band_in band
// rows (others zero).  Output rows likewise with band_out.
template <typename T, int N, int DIR>
__global__ void __launch_bounds__(256) k_colpass(const cx<T>* in, cx<T>* out, ColArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* A = tw + N;
  cx<T>* B = A + N * a.W;
  load_twiddles<T, N, DIR>(tw);
  const int tiles = a.ncols >> a.logW;
  const int64_t p = blockIdx.x / tiles;
  const int c0 = (blockIdx.x - (int)(p * tiles)) << a.logW;
  const cx<T>* src = in + p * a.plane_in + c0;
  for (int idx = threadIdx.x; idx < N * a.W; idx += blockDim.x) {
    const int r = idx >> a.logW, c = idx & (a.W - 1);
    int j = r;
    bool ok = true;
    if (a.band_in) {
      // band rows n = -(M-1) .. M-1; the unpaired n = -M row is read as zero so
      // that inverse transforms see a Hermitian-consistent kz = 0 plane
      if (r < a.band_in) j = r;
      else if (r > N - a.band_in) j = r - N + 2 * a.band_in;
      else ok = false;
    }
    if (ok && a.mask_m) {
      const int col = c0 + c;
      const int jy = col / a.mask_m, kz = col - jy * a.mask_m;
      const int nx = freq_of(r, N), ny = band_freq(jy, a.mask_m);
      const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)kz * kz;
      const int b = a.mask_b0 + (int)p;
      ok = n2 > 0 && n2 >= a.thr[b] && n2 < a.thr[b + 1] && nx != -(N / 2) && ny != -(N / 2) &&
           ny != -a.mask_m;
    }
    A[idx] = ok ? src[(int64_t)j * a.row_in + c] : cx<T>{T(0), T(0)};
  }
  __syncthreads();
  cx<T>* R = fft_lds<T, N, DIR, true>(A, B, a.W, a.logW, 1, a.W, tw);
  cx<T>* dst = out + p * a.plane_out + c0;
  for (int idx = threadIdx.x; idx < N * a.W; idx += blockDim.x) {
    const int r = idx >> a.logW, c = idx & (a.W - 1);
    int j = r;
    if (a.band_out) {
      if (r < a.band_out) j = r;
      else if (r >= N - a.band_out) j = r - N + 2 * a.band_out;
      else continue;
    }
    dst[(int64_t)j * a.row_out + c] = R[idx];
  }
}

// Column analogue of row_fft_q for N = R1 R2 (R2 = Q R1): W = 256 / R1
// columns x R1 ranks; lane (c, rank) holds rows rank + R1 n2 (n2 < R2) on
// entry and rows (rank + R1 i) + R2 k2 in v[i R1 + k2] on exit.  LDS layout
// [k1][n1][c] with 16 elements of padding per k1 block; two barriers.
template <typename T, int R1, int R2, int DIR>
__device__ __forceinline__ void col_fft_q(cx<T>* v, int c, int rank, cx<T>* buf, const cx<T>* tw) {
  constexpr int W = 256 / R1, Q = R2 / R1;
  dft_reg<T, R2, DIR>(v);
#pragma unroll
  for (int k1 = 0; k1 < R2; ++k1)
    buf[(k1 * R1 + rank) * W + c + 16 * k1] = k1 == 0 ? v[k1] : cmul(v[k1], tw[rank * k1]);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int k1 = rank + R1 * i;
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) v[i * R1 + n1] = buf[(k1 * R1 + n1) * W + c + 16 * k1];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i) dft_reg<T, R1, DIR>(v + i * R1);
}

// Column pass for N = R1 R2 with R2 = 2 R1 (N = 128, 512): same arguments,
// band and mask semantics as k_colpass.
template <typename T, int R1, int R2, int DIR>
__global__ void __launch_bounds__(256) k_colpass_q(const cx<T>* in, cx<T>* out, ColArgs a) {
  constexpr int N = R1 * R2, W = 256 / R1, Q = R2 / R1;
  constexpr int LOGW = (W == 8 ? 3 : W == 16 ? 4 : W == 32 ? 5 : 6);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;
  load_twiddles<T, N, DIR>(tw);
  const int c = threadIdx.x & (W - 1), rank = threadIdx.x >> LOGW;
  const int tiles = a.ncols >> LOGW;
  const int64_t p = blockIdx.x / tiles;
  const int c0 = (blockIdx.x - (int)(p * tiles)) << LOGW;
  const cx<T>* src = in + p * a.plane_in + c0 + c;
  int jy = 0, kz = 0;
  if (a.mask_m) {
    jy = (c0 + c) / a.mask_m;
    kz = (c0 + c) - jy * a.mask_m;
  }
  cx<T> v[R2];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    const int r = rank + R1 * n2;
    int j = r;
    bool ok = true;
    if (a.band_in) {
      if (r < a.band_in) j = r;
      else if (r > N - a.band_in) j = r - N + 2 * a.band_in;
      else ok = false;
    }
    if (ok && a.mask_m) {
      const int nx = freq_of(r, N), ny = band_freq(jy, a.mask_m);
      const int64_t n2s = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)kz * kz;
      const int b = a.mask_b0 + (int)p;
      ok = n2s > 0 && n2s >= a.thr[b] && n2s < a.thr[b + 1] && nx != -(N / 2) && ny != -(N / 2) &&
           ny != -a.mask_m;
    }
    v[n2] = ok ? src[(int64_t)j * a.row_in] : cx<T>{T(0), T(0)};
  }
  __syncthreads();  // twiddles
  col_fft_q<T, R1, R2, DIR>(v, c, rank, buf, tw);
  cx<T>* dst = out + p * a.plane_out + c0 + c;
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int k2 = 0; k2 < R1; ++k2) {
      const int r = rank + R1 * i + R2 * k2;
      int j = r;
      if (a.band_out) {
        if (r < a.band_out) j = r;
        else if (r >= N - a.band_out) j = r - N + 2 * a.band_out;
        else continue;
      }
      dst[(int64_t)j * a.row_out] = v[i * R1 + k2];
    }
}

// z-row c2r for N = R1 R2 (R2 = 2 R1): a group of R1 lanes per row pair;
// same layouts and semantics as k_zpass_c2r.
template <typename T, int R1, int R2>
__global__ void __launch_bounds__(256) k_zpass_c2r_q(const cx<T>* in, T* out, int64_t npairs, int kz_in) {
  constexpr int N = R1 * R2, GR = 256 / R1, Q = R2 / R1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T, N, 1>(tw);
  const int grp = threadIdx.x / R1, rank = threadIdx.x % R1;
  cx<T>* buf = tw + N + grp * (R2 * (R1 + 1));
  const int64_t q = (int64_t)blockIdx.x * GR + grp;
  const bool live = q < npairs;
  const cx<T>* r0 = in + 2 * q * (int64_t)kz_in;
  cx<T> v[R2];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
    const int k = rank + R1 * n2;
    cx<T> z = {T(0), T(0)};
    if (live) {
      if (k < (N >> 1)) {
        if (k < kz_in) {
          const cx<T> a = r0[k], b = r0[kz_in + k];
          z = cx<T>{a.x - b.y, a.y + b.x};
        }
      } else if (k > (N >> 1)) {
        const int kk = N - k;
        if (kk < kz_in) {
          const cx<T> a = r0[kk], b = r0[kz_in + kk];
          z = cx<T>{a.x + b.y, b.x - a.y};
        }
      }
    }
    v[n2] = z;
  }
  __syncthreads();
  row_fft_q<T, R1, R2, 1>(v, rank, buf, tw);
  if (live) {
    T* o = out + 2 * q * (int64_t)N;
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int k2 = 0; k2 < R1; ++k2) {
        const int e = rank + R1 * i + R2 * k2;
        o[e] = v[i * R1 + k2].x;
        o[N + e] = v[i * R1 + k2].y;
      }
  }
}

// Register column pass for N = R^2: 256 threads = W = 256 / R columns x R
// ranks.  Lane (c, rank) loads rows rank + R n2 of column c, does the first
// R-point DFT in registers, exchanges through LDS (layout [k1][n1][c] with 16
// elements of padding per k1 block, so that the stage-1 writes and the stage-2
// reads of a half wavefront hit distinct banks) and does the second R-point
// DFT; it then holds output rows rank + R k2.  Same arguments and band / mask
// semantics as k_colpass.
template <typename T, int R, int DIR>
__global__ void __launch_bounds__(256) k_colpass_rr(const cx<T>* in, cx<T>* out, ColArgs a) {
  constexpr int N = R * R, W = 256 / R, LOGW = (W == 8 ? 3 : W == 16 ? 4 : W == 32 ? 5 : 6);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;
  load_twiddles<T, N, DIR>(tw);
  const int c = threadIdx.x & (W - 1), rank = threadIdx.x >> LOGW;
  const int tiles = a.ncols >> LOGW;
  const int64_t p = blockIdx.x / tiles;
  const int c0 = (blockIdx.x - (int)(p * tiles)) << LOGW;
  const cx<T>* src = in + p * a.plane_in + c0 + c;
  int jy = 0, kz = 0;
  if (a.mask_m) {
    jy = (c0 + c) / a.mask_m;
    kz = (c0 + c) - jy * a.mask_m;
  }
  cx<T> v[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int r = rank + R * n2;
    int j = r;
    bool ok = true;
    if (a.band_in) {
      // band rows n = -(M-1) .. M-1; the unpaired n = -M row is read as zero
      if (r < a.band_in) j = r;
      else if (r > N - a.band_in) j = r - N + 2 * a.band_in;
      else ok = false;
    }
    if (ok && a.mask_m) {
      const int nx = freq_of(r, N), ny = band_freq(jy, a.mask_m);
      const int64_t n2s = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)kz * kz;
      const int b = a.mask_b0 + (int)p;
      ok = n2s > 0 && n2s >= a.thr[b] && n2s < a.thr[b + 1] && nx != -(N / 2) && ny != -(N / 2) &&
           ny != -a.mask_m;
    }
    v[n2] = ok ? src[(int64_t)j * a.row_in] : cx<T>{T(0), T(0)};
  }
  __syncthreads();  // twiddles
  col_fft_rr<T, R, DIR>(v, c, rank, buf, tw);
  cx<T>* dst = out + p * a.plane_out + c0 + c;
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) {
    const int r = rank + R * k2;
    int j = r;
    if (a.band_out) {
      if (r < a.band_out) j = r;
      else if (r >= N - a.band_out) j = r - N + 2 * a.band_out;
      else continue;
    }
    dst[(int64_t)j * a.row_out] = v[k2];
  }
}

// Fused x pass of the interlaced full transform (N = R^2): for W columns
// (iy, kz) of both phase spectra (after their z and y passes, layout
// [phase][x][y][kz < N/2]) the forward x transforms of A and B, the combination
// D = 1/2 [A + e^{-i pi (nx + ny + kz) / N} B] (D = 0 on a Nyquist row or
// column), the band copy of D (-mb <= nx, ny < mb, kz < mb), and the inverse x
// transform of scale * D, written to out (layout [x][y][kz]).
template <typename T, int R>
__global__ void __launch_bounds__(256) k_xpass_interlace_rr(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                            cx<T>* __restrict__ band_out, int mb, T scale) {
  constexpr int N = R * R, W = 256 / R, H = N / 2;
  constexpr int LOGW = (W == 8 ? 3 : W == 16 ? 4 : W == 32 ? 5 : 6);
  constexpr int64_t ROW = (int64_t)N * H, PHASE = (int64_t)N * N * H;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* twf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twi = twf + N;
  cx<T>* tph = twi + N;  // [2N]: exp(-i pi s / N), the interlacing phase of nx + ny + kz = s (mod 2N)
  cx<T>* buf = tph + 2 * N;
  load_twiddles<T, N, -1>(twf);
  load_twiddles<T, N, 1>(twi);
  for (int t = threadIdx.x; t < 2 * N; t += blockDim.x) {
    const cx<double> w = g_twiddle1024[t * (512 / N)];
    tph[t] = cx<T>{T(w.x), T(w.y)};
  }
  const int c = threadIdx.x & (W - 1), rank = threadIdx.x >> LOGW;
  const int col = blockIdx.x * W + c;
  cx<T> va[R], vb[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int64_t o = (int64_t)(rank + R * n2) * ROW + col;
    va[n2] = in[o];
    vb[n2] = in[PHASE + o];
  }
  __syncthreads();  // twiddles
  col_fft_rr<T, R, -1>(va, c, rank, buf, twf);
  col_fft_rr<T, R, -1>(vb, c, rank, buf, twf);
  const int iy = col / H, kz = col - iy * H;
  const int ny = iy < H ? iy : iy - N;
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) {
    const int row = rank + R * k2;
    const int nx = row < H ? row : row - N;
    cx<T> d = {T(0), T(0)};
    if (nx != -H && ny != -H) d = cscale(cadd(va[k2], cmul(tph[(nx + ny + kz) & (2 * N - 1)], vb[k2])), T(0.5));
    if (band_out && nx >= -mb && nx < mb && ny >= -mb && ny < mb && kz < mb) {
      const int bx = nx < 0 ? nx + 2 * mb : nx, by = ny < 0 ? ny + 2 * mb : ny;
      band_out[((int64_t)bx * 2 * mb + by) * mb + kz] = d;
    }
    va[k2] = cscale(d, scale);
  }
  col_fft_rr<T, R, 1>(va, c, rank, buf, twi);
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) out[(int64_t)(rank + R * k2) * ROW + col] = va[k2];
}

template <typename T>
cnpc_status xpass_interlace(int n, const cx<T>* in, cx<T>* out, cx<T>* band_out, int mb, T scale,
                            hipStream_t s) {
  auto go = [&](auto rc) -> cnpc_status {
    constexpr int R = decltype(rc)::value, N = R * R, W = 256 / R;
    const int64_t cols = (int64_t)N * (N / 2);
    const size_t lds = sizeof(cx<T>) * (4 * N + (size_t)N * W + 16 * R);
    kt_begin(CNPC_KT_COL, s);
    hipLaunchKernelGGL((k_xpass_interlace_rr<T, R>), dim3((unsigned)(cols / W)), dim3(256), lds, s, in, out,
                       band_out, mb, scale);
    kt_end(CNPC_KT_COL, s);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  };
  if (n == 64) return go(std::integral_constant<int, 8>());
  if (n == 256) return go(std::integral_constant<int, 16>());
  set_error("fused interlace pass needs N = 64 or 256 (got %d)", n);
  return CNPC_EUNSUPPORTED;
}
template cnpc_status xpass_interlace<float>(int, const cx<float>*, cx<float>*, cx<float>*, int, float,
                                            hipStream_t);
template cnpc_status xpass_interlace<double>(int, const cx<double>*, cx<double>*, cx<double>*, int, double,
                                             hipStream_t);

// ------------------------------------------------------------- launchers --
// side R of the register passes for N = R^2 (0: LDS Stockham passes)
constexpr int rr_radix(int n) { return n == 64 ? 8 : n == 256 ? 16 : 0; }

template <typename T, int N>
static cnpc_status zr2c_n(const T* in, cx<T>* out, int64_t nrows, int kz, hipStream_t s) {
  const int64_t npairs = nrows / 2;
  constexpr int R = rr_radix(N);
  if constexpr (R > 0) if (fft_register_passes()) {
    constexpr int GR = 256 / R;
    const size_t lds = sizeof(cx<T>) * (N + (size_t)GR * R * (R + 1));
    kt_begin(CNPC_KT_ZR2C, s);
    hipLaunchKernelGGL((k_zpass_r2c_rr<T, R>), dim3((unsigned)((npairs + GR - 1) / GR)), dim3(256), lds, s, in,
                       out, npairs, kz);
    kt_end(CNPC_KT_ZR2C, s);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  }
  constexpr int NSEQ = ZCfg<T, N>::NSEQ;
  const int64_t blocks = (npairs + NSEQ - 1) / NSEQ;
  const size_t lds = sizeof(cx<T>) * (N + 2 * NSEQ * N);
  kt_begin(CNPC_KT_ZR2C, s);
  hipLaunchKernelGGL((k_zpass_r2c<T, N>), dim3((unsigned)blocks), dim3(256), lds, s, in, out, npairs,
                     kz);
  kt_end(CNPC_KT_ZR2C, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// R1 of the N = R1 (2 R1) register passes (0: none)
constexpr int q_radix(int n) { return n == 128 ? 8 : n == 512 ? 16 : 0; }

template <typename T, int N>
static cnpc_status zc2r_n(const cx<T>* in, T* out, int64_t nrows, int kz, hipStream_t s) {
  const int64_t npairs = nrows / 2;
  constexpr int R1 = q_radix(N);
  if constexpr (R1 > 0) if (fft_register_passes()) {
    constexpr int R2 = 2 * R1, GR = 256 / R1;
    const size_t lds = sizeof(cx<T>) * (N + (size_t)GR * R2 * (R1 + 1));
    kt_begin(CNPC_KT_ZC2R, s);
    hipLaunchKernelGGL((k_zpass_c2r_q<T, R1, R2>), dim3((unsigned)((npairs + GR - 1) / GR)), dim3(256), lds, s,
                       in, out, npairs, kz);
    kt_end(CNPC_KT_ZC2R, s);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  }
  constexpr int R = rr_radix(N);
  if constexpr (R > 0) if (fft_register_passes()) {
    constexpr int GR = 256 / R;
    const size_t lds = sizeof(cx<T>) * (N + (size_t)GR * R * (R + 1));
    kt_begin(CNPC_KT_ZC2R, s);
    hipLaunchKernelGGL((k_zpass_c2r_rr<T, R>), dim3((unsigned)((npairs + GR - 1) / GR)), dim3(256), lds, s, in,
                       out, npairs, kz);
    kt_end(CNPC_KT_ZC2R, s);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  }
  constexpr int NSEQ = ZCfg<T, N>::NSEQ;
  const int64_t blocks = (npairs + NSEQ - 1) / NSEQ;
  const size_t lds = sizeof(cx<T>) * (N + 2 * NSEQ * N);
  kt_begin(CNPC_KT_ZC2R, s);
  hipLaunchKernelGGL((k_zpass_c2r<T, N>), dim3((unsigned)blocks), dim3(256), lds, s, in, out, npairs,
                     kz);
  kt_end(CNPC_KT_ZC2R, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

template <typename T, int N, int DIR>
static cnpc_status col_n(const cx<T>* in, cx<T>* out, const ColArgs& a, int64_t nplanes,
                         hipStream_t s) {
  constexpr int R1 = q_radix(N);
  if constexpr (R1 > 0) {
    constexpr int R2 = 2 * R1, W = 256 / R1;
    if (a.ncols % W == 0 && fft_register_passes()) {
      const int64_t blocks = nplanes * (a.ncols / W);
      if (blocks <= 0) return CNPC_OK;
      if (blocks > 0x7fffffffLL) {
        set_error("column pass grid too large");
        return CNPC_EUNSUPPORTED;
      }
      const size_t lds = sizeof(cx<T>) * (N + (size_t)N * W + 16 * R2);
      kt_begin(CNPC_KT_COL, s);
      hipLaunchKernelGGL((k_colpass_q<T, R1, R2, DIR>), dim3((unsigned)blocks), dim3(256), lds, s, in, out, a);
      kt_end(CNPC_KT_COL, s);
      CNPC_HIP(hipGetLastError());
      return CNPC_OK;
    }
  }
  constexpr int R = rr_radix(N);
  if constexpr (R > 0) {
    constexpr int W = 256 / R;
    if (a.ncols % W == 0 && fft_register_passes()) {
      const int64_t blocks = nplanes * (a.ncols / W);
      if (blocks <= 0) return CNPC_OK;
      if (blocks > 0x7fffffffLL) {
        set_error("column pass grid too large");
        return CNPC_EUNSUPPORTED;
      }
      const size_t lds = sizeof(cx<T>) * (N + (size_t)N * W + 16 * R);
      kt_begin(CNPC_KT_COL, s);
      hipLaunchKernelGGL((k_colpass_rr<T, R, DIR>), dim3((unsigned)blocks), dim3(256), lds, s, in, out, a);
      kt_end(CNPC_KT_COL, s);
      CNPC_HIP(hipGetLastError());
      return CNPC_OK;
    }
  }
  const int64_t blocks = nplanes * (a.ncols >> a.logW);
  if (blocks <= 0) return CNPC_OK;
  if (blocks > 0x7fffffffLL) {
    set_error("column pass grid too large");
    return CNPC_EUNSUPPORTED;
  }
  const size_t lds = sizeof(cx<T>) * (N + 2 * N * a.W);
  kt_begin(CNPC_KT_COL, s);
  hipLaunchKernelGGL((k_colpass<T, N, DIR>), dim3((unsigned)blocks), dim3(256), lds, s, in, out, a);
  kt_end(CNPC_KT_COL, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

#define CNPC_DISPATCH_N(n, CALL)          \
  switch (n) {                            \
    case 16: { constexpr int NN = 16; return CALL; }     \
    case 32: { constexpr int NN = 32; return CALL; }     \
    case 64: { constexpr int NN = 64; return CALL; }     \
    case 128: { constexpr int NN = 128; return CALL; }   \
    case 256: { constexpr int NN = 256; return CALL; }   \
    case 512: { constexpr int NN = 512; return CALL; }   \
    case 1024: { constexpr int NN = 1024; return CALL; } \
    default: set_error("unsupported mesh size %d", n); return CNPC_EUNSUPPORTED; \
  }

template <typename T>
cnpc_status zpass_r2c(int n, const T* in, cx<T>* out, int64_t nrows, int kz, hipStream_t s) {
  CNPC_DISPATCH_N(n, (zr2c_n<T, NN>(in, out, nrows, kz, s)));
}
template <typename T>
cnpc_status zpass_c2r(int n, const cx<T>* in, T* out, int64_t nrows, int kz, hipStream_t s) {
  CNPC_DISPATCH_N(n, (zc2r_n<T, NN>(in, out, nrows, kz, s)));
}
template <typename T>
cnpc_status colpass(int n, int dir, const cx<T>* in, cx<T>* out, const ColArgs& a, int64_t nplanes,
                    hipStream_t s) {
  if (dir < 0) {
    CNPC_DISPATCH_N(n, (col_n<T, NN, -1>(in, out, a, nplanes, s)));
  }
  CNPC_DISPATCH_N(n, (col_n<T, NN, 1>(in, out, a, nplanes, s)));
}

ColArgs make_col(int n, int dtype, int64_t plane_in, int64_t plane_out, int64_t row_in,
                 int64_t row_out, int ncols, int band_in, int band_out) {
  ColArgs a;
  a.plane_in = plane_in;
  a.plane_out = plane_out;
  a.row_in = row_in;
  a.row_out = row_out;
  a.ncols = ncols;
  int w = col_tile_width(n, dtype);
  while (w > 1 && (ncols % w) != 0) w >>= 1;
  a.W = w;
  a.logW = ilog2_host(w);
  a.band_in = band_in;
  a.band_out = band_out;
  a.mask_m = 0;
  a.mask_b0 = 0;
  return a;
}

// ------------------------------------------------------- 3-D transforms --
template <typename T>
cnpc_status fft3d_r2c(int n, int batch, int band, const T* in, cx<T>* out, cx<T>* ws,
                      hipStream_t s) {
  CNPC_TRY(ensure_twiddles());
  const int dt = sizeof(T) == 8 ? CNPC_F64 : CNPC_F32;
  const int64_t nn = (int64_t)n * n;
  if (band == 0) {
    const int h = n / 2;
    CNPC_TRY(zpass_r2c<T>(n, in, out, (int64_t)batch * nn, h, s));
    // y: planes (b, ix), rows iy (stride h), columns kz
    ColArgs ay = make_col(n, dt, (int64_t)n * h, (int64_t)n * h, h, h, h, 0, 0);
    CNPC_TRY(colpass<T>(n, -1, out, out, ay, (int64_t)batch * n, s));
    // x: planes b, rows ix (stride n*h), columns (iy, kz)
    ColArgs ax = make_col(n, dt, nn * h, nn * h, (int64_t)n * h, (int64_t)n * h, n * h, 0, 0);
    CNPC_TRY(colpass<T>(n, -1, out, out, ax, batch, s));
    return CNPC_OK;
  }
  const int m = band;
  cx<T>* w1 = ws;                              // [batch][n][n][m]
  cx<T>* w2 = ws + (int64_t)batch * nn * m;    // [batch][n][2m][m]
  CNPC_TRY(zpass_r2c<T>(n, in, w1, (int64_t)batch * nn, m, s));
  ColArgs ay = make_col(n, dt, (int64_t)n * m, (int64_t)2 * m * m, m, m, m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, w1, w2, ay, (int64_t)batch * n, s));
  ColArgs ax = make_col(n, dt, (int64_t)n * 2 * m * m, (int64_t)4 * m * m * m, (int64_t)2 * m * m,
                        (int64_t)2 * m * m, 2 * m * m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, w2, out, ax, batch, s));
  return CNPC_OK;
}

template <typename T>
cnpc_status fft3d_c2r(int n, int batch, int band, const cx<T>* in, T* out, cx<T>* ws,
                      hipStream_t s) {
  CNPC_TRY(ensure_twiddles());
  const int dt = sizeof(T) == 8 ? CNPC_F64 : CNPC_F32;
  const int64_t nn = (int64_t)n * n;
  if (band == 0) {
    const int h = n / 2;
    cx<T>* o = reinterpret_cast<cx<T>*>(out);
    ColArgs ax = make_col(n, dt, nn * h, nn * h, (int64_t)n * h, (int64_t)n * h, n * h, 0, 0);
    CNPC_TRY(colpass<T>(n, 1, in, o, ax, batch, s));
    ColArgs ay = make_col(n, dt, (int64_t)n * h, (int64_t)n * h, h, h, h, 0, 0);
    CNPC_TRY(colpass<T>(n, 1, o, o, ay, (int64_t)batch * n, s));
    CNPC_TRY(zpass_c2r<T>(n, o, out, (int64_t)batch * nn, h, s));
    return CNPC_OK;
  }
  const int m = band;
  cx<T>* w1 = ws;                            // [batch][n][n][m]
  cx<T>* w2 = ws + (int64_t)batch * nn * m;  // [batch][n][2m][m]
  ColArgs ax = make_col(n, dt, (int64_t)4 * m * m * m, (int64_t)n * 2 * m * m, (int64_t)2 * m * m,
                        (int64_t)2 * m * m, 2 * m * m, m, 0);
  CNPC_TRY(colpass<T>(n, 1, in, w2, ax, batch, s));
  ColArgs ay = make_col(n, dt, (int64_t)2 * m * m, (int64_t)n * m, m, m, m, m, 0);
  CNPC_TRY(colpass<T>(n, 1, w2, w1, ay, (int64_t)batch * n, s));
  CNPC_TRY(zpass_c2r<T>(n, w1, out, (int64_t)batch * nn, m, s));
  return CNPC_OK;
}

size_t fft_ws_elems(int n, int batch, int band) {
  if (band == 0) return 0;
  const size_t nn = (size_t)n * n;
  return (size_t)batch * (nn * band + (size_t)n * 2 * band * band);
}

template cnpc_status zpass_r2c<float>(int, const float*, cx<float>*, int64_t, int, hipStream_t);
template cnpc_status zpass_r2c<double>(int, const double*, cx<double>*, int64_t, int, hipStream_t);
template cnpc_status zpass_c2r<float>(int, const cx<float>*, float*, int64_t, int, hipStream_t);
template cnpc_status zpass_c2r<double>(int, const cx<double>*, double*, int64_t, int, hipStream_t);
template cnpc_status colpass<float>(int, int, const cx<float>*, cx<float>*, const ColArgs&, int64_t,
                                    hipStream_t);
template cnpc_status colpass<double>(int, int, const cx<double>*, cx<double>*, const ColArgs&,
                                     int64_t, hipStream_t);
template cnpc_status fft3d_r2c<float>(int, int, int, const float*, cx<float>*, cx<float>*,
                                      hipStream_t);
template cnpc_status fft3d_r2c<double>(int, int, int, const double*, cx<double>*, cx<double>*,
                                       hipStream_t);
template cnpc_status fft3d_c2r<float>(int, int, int, const cx<float>*, float*, cx<float>*,
                                      hipStream_t);
template cnpc_status fft3d_c2r<double>(int, int, int, const cx<double>*, double*, cx<double>*,
                                       hipStream_t);

}  // namespace cnpc
