// LDS-staged radix-8/4 Stockham FFT building blocks for 64-wide wavefronts.
//
// A workgroup transforms `nseq` independent length-N sequences that sit in
// LDS (element e of sequence s at buf[s * sstride + e * estride]).  Each stage
// reads R strided values per task into registers, applies the twiddles
// w^(r k), does an R-point DFT in registers and writes the autosorted result
// to the other LDS buffer (ping-pong, one barrier per stage).  Radix-8 stages
// first, then radix-4: N = 8^a 4^b.
#pragma once

#include "common.h"

namespace cnpc {

// exp(-2 pi i t / 1024), t = 0..1023, FP64; set once per device by the host.
extern __device__ cx<double> g_twiddle1024[1024];

template <int N>
struct Radix {
  static constexpr int L = (N <= 1) ? 0 : 1 + Radix<N / 2>::L;
  static constexpr int n8 = (L % 3 == 0) ? L / 3 : ((L % 3 == 1) ? (L - 4) / 3 : (L - 2) / 3);
  static constexpr int n4 = (L - 3 * n8) / 2;
};
template <>
struct Radix<1> {
  static constexpr int L = 0;
  static constexpr int n8 = 0;
  static constexpr int n4 = 0;
};

// multiply by DIR * i (DIR = -1: forward, -i; DIR = +1: inverse, +i)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return DIR < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
  const cx<T> t3 = mul_i<T, DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft8(cx<T>* v) {
  dft4<T, DIR>(v[0], v[2], v[4], v[6]);  // E0..E3
  dft4<T, DIR>(v[1], v[3], v[5], v[7]);  // O0..O3
  const T r = T(0.70710678118654752440);
  const cx<T> o0 = v[1];
  cx<T> o1 = v[3], o2 = v[5], o3 = v[7];
  if (DIR < 0) {  // W = exp(-i pi/4)
    o1 = {r * (o1.x + o1.y), r * (o1.y - o1.x)};
    o2 = {o2.y, -o2.x};
    o3 = {r * (o3.y - o3.x), -r * (o3.x + o3.y)};
  } else {  // W = exp(+i pi/4)
    o1 = {r * (o1.x - o1.y), r * (o1.x + o1.y)};
    o2 = {-o2.y, o2.x};
    o3 = {-r * (o3.x + o3.y), r * (o3.x - o3.y)};
  }
  const cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 8) {
    dft8<T, DIR>(v);
  } else {
    dft4<T, DIR>(v[0], v[1], v[2], v[3]);
  }
}

// cos(2 pi j / 32) from the first-octant values and quadrant symmetry.
__host__ __device__ constexpr double cos_frac32(int j) {
  j &= 31;
  constexpr double c8[9] = {1.0,
                            0.98078528040323044913,
                            0.92387953251128675613,
                            0.83146961230254523708,
                            0.70710678118654752440,
                            0.55557023301960222474,
                            0.38268343236508977173,
                            0.19509032201612826785,
                            0.0};
  return j <= 8 ? c8[j] : (j <= 16 ? -c8[16 - j] : (j <= 24 ? -c8[j - 16] : c8[32 - j]));
}

// W_R^j = exp(DIR 2 pi i j / R) for R dividing 32
template <typename T, int R, int DIR>
__device__ __forceinline__ cx<T> wR(int j) {
  const int q = (j * (32 / R)) & 31;
  return cx<T>{T(cos_frac32(q)), T(DIR * cos_frac32(q - 8))};
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cx<T>* v);

// R = P Q point DFT of registers, natural order in and out: n = a + P b,
// k = c + Q d; Q-point DFTs over b, twiddles W_R^(a c), P-point DFTs over a.
template <typename T, int P, int Q, int DIR>
__device__ __forceinline__ void dft_composite(cx<T>* v) {
  constexpr int R = P * Q;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    cx<T> t[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) t[b] = v[a + P * b];
    dft_reg<T, Q, DIR>(t);
#pragma unroll
    for (int c = 0; c < Q; ++c) v[a + P * c] = (a * c == 0) ? t[c] : cmul(t[c], wR<T, R, DIR>(a * c));
  }
  cx<T> o[R];
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    cx<T> t[P];
#pragma unroll
    for (int a = 0; a < P; ++a) t[a] = v[a + P * c];
    dft_reg<T, P, DIR>(t);
#pragma unroll
    for (int d = 0; d < P; ++d) o[c + Q * d] = t[d];
  }
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = o[k];
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cx<T>* v) {
  if constexpr (R == 2) {
    const cx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else if constexpr (R == 4) {
    dft4<T, DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<T, DIR>(v);
  } else if constexpr (R == 16) {
    dft_composite<T, 4, 4, DIR>(v);
  } else {
    static_assert(R == 32, "register DFT sizes: 2, 4, 8, 16, 32");
    dft_composite<T, 4, 8, DIR>(v);
  }
}

// Orders the LDS accesses of one wavefront around an exchange among its own
// lanes: the LDS executes a wavefront's operations in issue order, so only the
// compiler has to be kept from moving accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Length N = R * R transform of one sequence by a group of R lanes (rank =
// lane within the group): on entry lane n1 holds x[n1 + R n2] in v[n2]; on
// exit it holds X[n1 + R k2] in v[k2].  Two register DFTs with one LDS
// transpose in between (buffer of R (R + 1) elements per group, padded so that
// both the row writes and the column reads are bank-conflict free); tw is the
// N-entry table W_N^t.  WAVE = false: two workgroup barriers, every lane of the
// workgroup must call it; WAVE = true: the group's buffer is its own and the
// group lies within one wavefront (R divides 64), and the transpose is ordered
// by wavefront-level syncs only (the caller has made tw visible).
template <typename T, int R, int DIR, bool WAVE = false>
__device__ __forceinline__ void row_fft_rr(cx<T>* v, int rank, cx<T>* buf, const cx<T>* tw) {
  static_assert(!WAVE || 64 % R == 0, "a wavefront-synchronised group lies within one wavefront");
  dft_reg<T, R, DIR>(v);  // lane n1: Y[n1][k1] in v[k1]
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) buf[k1 * (R + 1) + rank] = k1 == 0 ? v[k1] : cmul(v[k1], tw[rank * k1]);
  if constexpr (WAVE) wave_lds_sync();
  else __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) v[n1] = buf[rank * (R + 1) + n1];
  if constexpr (WAVE) wave_lds_sync();
  else __syncthreads();
  dft_reg<T, R, DIR>(v);
}

// Length N = R^2 transform of W = 256 / R columns by a workgroup: lane (c,
// rank) holds rows rank + R n2 of column c in v[n2] on entry and rows
// rank + R k2 of the transform in v[k2] on exit.  One LDS exchange (layout
// [k1][n1][c], 16 elements of padding per k1 block, conflict free for the
// stage-1 writes and the stage-2 reads of a half wavefront); contains one
// workgroup barrier before the exchange reads and one after them.
template <typename T, int R, int DIR>
__device__ __forceinline__ void col_fft_rr(cx<T>* v, int c, int rank, cx<T>* buf, const cx<T>* tw) {
  constexpr int W = 256 / R;
  dft_reg<T, R, DIR>(v);
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1)
    buf[(k1 * R + rank) * W + c + 16 * k1] = k1 == 0 ? v[k1] : cmul(v[k1], tw[rank * k1]);
  __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < R; ++n1) v[n1] = buf[(rank * R + n1) * W + c + 16 * rank];
  __syncthreads();
  dft_reg<T, R, DIR>(v);
}

// Length N = R1 R2 transform (R2 = Q R1) of one sequence by a group of R1
// lanes: on entry lane n1 holds x[n1 + R1 n2] in v[n2] (n2 < R2); on exit it
// holds X[(n1 + R1 i) + R2 k2] in v[i R1 + k2] (i < Q, k2 < R1).  R2-point
// register DFTs, one padded LDS exchange (R2 (R1 + 1) elements per group), Q
// R1-point register DFTs per lane.  Two workgroup barriers.
template <typename T, int R1, int R2, int DIR>
__device__ __forceinline__ void row_fft_q(cx<T>* v, int rank, cx<T>* buf, const cx<T>* tw) {
  constexpr int Q = R2 / R1;
  dft_reg<T, R2, DIR>(v);  // lane n1: Y[n1][k1] in v[k1]
#pragma unroll
  for (int k1 = 0; k1 < R2; ++k1) buf[k1 * (R1 + 1) + rank] = k1 == 0 ? v[k1] : cmul(v[k1], tw[rank * k1]);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) v[i * R1 + n1] = buf[(rank + R1 * i) * (R1 + 1) + n1];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i) dft_reg<T, R1, DIR>(v + i * R1);
}

// Twiddle table tw[t] = exp(DIR 2 pi i t / N) into LDS.
template <typename T, int N, int DIR>
__device__ __forceinline__ void load_twiddles(cx<T>* tw) {
  constexpr int step = 1024 / N;
  for (int t = threadIdx.x; t < N; t += blockDim.x) {
    const cx<double> w = g_twiddle1024[t * step];
    tw[t] = cx<T>{T(w.x), DIR < 0 ? T(w.y) : T(-w.y)};
  }
}

// One Stockham stage, src -> dst.  SEQ_FAST: consecutive tasks walk the
// sequences (column layouts, nseq a power of two = 1 << lognseq); otherwise
// they walk the elements of one sequence (row layouts).
template <typename T, int N, int R, int DIR, bool SEQ_FAST>
__device__ __forceinline__ void fft_stage(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                          int nseq, int lognseq, int sstride, int estride,
                                          const cx<T>* __restrict__ tw, int Ns) {
  constexpr int per = N / R;
  const int tasks = nseq * per;
  for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
    int s, j;
    if constexpr (SEQ_FAST) {
      s = task & (nseq - 1);
      j = task >> lognseq;
    } else {
      s = task / per;
      j = task - s * per;
    }
    const cx<T>* in = src + s * sstride;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[(j + r * per) * estride];
    const int k = j & (Ns - 1);
    if (Ns > 1) {
      const int step = (N / (Ns * R)) * k;
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * step]);
    }
    dftR<T, R, DIR>(v);
    const int base = (j - k) * R + k;
    cx<T>* out = dst + s * sstride;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(base + r * Ns) * estride] = v[r];
  }
}

// Full FFT of all sequences; data must be in `a` and visible (barrier done).
// Returns the buffer that holds the result; ends with a barrier.
template <typename T, int N, int DIR, bool SEQ_FAST>
__device__ __forceinline__ cx<T>* fft_lds(cx<T>* a, cx<T>* b, int nseq, int lognseq, int sstride,
                                          int estride, const cx<T>* tw) {
  cx<T>* src = a;
  cx<T>* dst = b;
  int Ns = 1;
#pragma unroll
  for (int i = 0; i < Radix<N>::n8; ++i) {
    fft_stage<T, N, 8, DIR, SEQ_FAST>(src, dst, nseq, lognseq, sstride, estride, tw, Ns);
    __syncthreads();
    cx<T>* t = src;
    src = dst;
    dst = t;
    Ns *= 8;
  }
#pragma unroll
  for (int i = 0; i < Radix<N>::n4; ++i) {
    fft_stage<T, N, 4, DIR, SEQ_FAST>(src, dst, nseq, lognseq, sstride, estride, tw, Ns);
    __syncthreads();
    cx<T>* t = src;
    src = dst;
    dst = t;
    Ns *= 4;
  }
  return src;
}

}  // namespace cnpc
