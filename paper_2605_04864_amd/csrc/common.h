// Shared device/host helpers of the cnpc library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/cnpc.h"

namespace cnpc {

// ---------------------------------------------------------------- errors --
void set_error(const char* fmt, ...);
void clear_error();

#define CNPC_REQUIRE(cond, ...)            \
  do {                                     \
    if (!(cond)) {                         \
      ::cnpc::set_error(__VA_ARGS__);      \
      return CNPC_EINVAL;                  \
    }                                      \
  } while (0)

#define CNPC_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::cnpc::set_error("HIP error %s at %s:%d", hipGetErrorString(e_), __FILE__, __LINE__); \
      return CNPC_EHIP;                                                             \
    }                                                                               \
  } while (0)

#define CNPC_TRY(call)              \
  do {                              \
    cnpc_status s_ = (call);        \
    if (s_ != CNPC_OK) return s_;   \
  } while (0)

// kernel timer hooks (no-ops unless cnpc_ktimer_start selected the class)
void kt_begin(int cls, hipStream_t s);
void kt_end(int cls, hipStream_t s);

// current value of a tuning knob (0: library default)
int tune_value(int knob);
// register FFT passes allowed (CNPC_TUNE_FFT_PASSES != 1)
inline bool fft_register_passes() { return tune_value(CNPC_TUNE_FFT_PASSES) != 1; }

cnpc_status check_desc(const cnpc_mesh_desc* d);
cnpc_status check_bins(const cnpc_mesh_desc* d, const cnpc_kbins* b);
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int ilog2_host(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }
inline size_t esize(int dtype) { return dtype == CNPC_F64 ? 8 : 4; }
// FP64 bin thresholds T_b = ceil(((kmin + b dk)/kf)^2), b = 0..nbins (host);
// an edge within a relative 1e-9 of an integer n^2 is taken to be on it
void bin_thresholds(const cnpc_mesh_desc* d, const cnpc_kbins* b, int64_t* out);

// ---------------------------------------------------------------- complex --
template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// wavenumber index of storage index i along an axis of length n (FFT order)
__device__ __forceinline__ int freq_of(int i, int n) { return i < (n >> 1) ? i : i - n; }
// wavenumber index of band storage index j (band half-width m)
__device__ __forceinline__ int band_freq(int j, int m) { return j < m ? j : j - 2 * m; }

// ------------------------------------------------- Racah spherical harmonics --
// y_l^m(u) = sqrt(4 pi/(2l+1)) Y_l^m(u) for a unit vector u = (x, y, z), m >= 0,
// Condon-Shortley phase.  Written as Cartesian polynomials of z and s = x + i y:
//   l=1: y10 = z,  y11 = -s/sqrt2
//   l=2: y20 = (3z^2-1)/2, y21 = -sqrt(3/2) s z, y22 = sqrt(3/8) s^2
//   l=3: y30 = (5z^3-3z)/2, y31 = -sqrt(3)/4 s (5z^2-1), y32 = sqrt(15/8) s^2 z,
//        y33 = -sqrt(5)/4 s^3
//   l=4: y40 = (35z^4-30z^2+3)/8, y41 = -sqrt(5)/4 s z (7z^2-3),
//        y42 = sqrt(5/2)/4 s^2 (7z^2-1), y43 = -sqrt(35)/4 s^3 z,
//        y44 = sqrt(35/2)/8 s^4
// (these follow from Y_l^m = (-1)^m sqrt((2l+1)/4pi (l-m)!/(l+m)!) P_l^m e^{i m phi}
// with P_l^m the associated Legendre function without the Condon-Shortley sign).
// Output: re[m], im[m] for m = 0..l.
template <typename T>
__device__ __forceinline__ void racah_ylm(int ell, T x, T y, T z, T* re, T* im) {
  const T s1r = x, s1i = y;                                  // s
  const T s2r = x * x - y * y, s2i = T(2) * x * y;           // s^2
  const T s3r = s2r * x - s2i * y, s3i = s2r * y + s2i * x;  // s^3
  const T s4r = s2r * s2r - s2i * s2i, s4i = T(2) * s2r * s2i;
  const T z2 = z * z;
  switch (ell) {
    case 0:
      re[0] = T(1); im[0] = T(0);
      break;
    case 1: {
      const T c = T(-0.70710678118654752440);
      re[0] = z; im[0] = T(0);
      re[1] = c * s1r; im[1] = c * s1i;
      break;
    }
    case 2: {
      re[0] = T(0.5) * (T(3) * z2 - T(1)); im[0] = T(0);
      const T c1 = T(-1.22474487139158904910) * z;  // -sqrt(3/2) z
      re[1] = c1 * s1r; im[1] = c1 * s1i;
      const T c2 = T(0.61237243569579452455);  // sqrt(3/8)
      re[2] = c2 * s2r; im[2] = c2 * s2i;
      break;
    }
    case 3: {
      re[0] = T(0.5) * z * (T(5) * z2 - T(3)); im[0] = T(0);
      const T c1 = T(-0.43301270189221932338) * (T(5) * z2 - T(1));  // -sqrt3/4
      re[1] = c1 * s1r; im[1] = c1 * s1i;
      const T c2 = T(1.36930639376291528364) * z;  // sqrt(15/8)
      re[2] = c2 * s2r; im[2] = c2 * s2i;
      const T c3 = T(-0.55901699437494742410);  // -sqrt5/4
      re[3] = c3 * s3r; im[3] = c3 * s3i;
      break;
    }
    default: {  // 4
      re[0] = T(0.125) * (T(35) * z2 * z2 - T(30) * z2 + T(3)); im[0] = T(0);
      const T c1 = T(-0.55901699437494742410) * z * (T(7) * z2 - T(3));  // -sqrt5/4
      re[1] = c1 * s1r; im[1] = c1 * s1i;
      const T c2 = T(0.39528470752104741650) * (T(7) * z2 - T(1));  // sqrt(5/2)/4
      re[2] = c2 * s2r; im[2] = c2 * s2i;
      const T c3 = T(-1.47901994577490951707) * z;  // -sqrt(35)/4
      re[3] = c3 * s3r; im[3] = c3 * s3i;
      const T c4 = T(0.52291251658379721749);  // sqrt(35/2)/8
      re[4] = c4 * s4r; im[4] = c4 * s4i;
      break;
    }
  }
}

// sinc(pi n / N)^p for the mass-assignment compensation, in FP64
__device__ __forceinline__ double window_1d(int n, int nmesh, int p) {
  if (n == 0) return 1.0;
  const double a = (double)n / (double)nmesh;
  const double s = sinpi(a) / (3.14159265358979323846 * a);
  double w = s * s;
  if (p == 3) w *= s;
  return w;
}

// alias sums of the squared 1-D window: c = sum_n W1^2(q + 2kN n) and the
// alternating c~ = sum_n (-1)^n W1^2(q + 2kN n), x = q H / 2 = pi n / N.
//   CIC: c = 1 - 2/3 sin^2 x,  c~ = cos x (5 + cos^2 x) / 6
//   TSC: c = 1 - sin^2 x + 2/15 sin^4 x,  c~ = cos x (cos^4 x + 58 cos^2 x + 61) / 120
__device__ __forceinline__ void alias_1d(int n, int nmesh, int p, double* c, double* ct) {
  const double a = (double)n / (double)nmesh;
  const double sx = sinpi(a), cxv = cospi(a);
  const double s2 = sx * sx, c2 = cxv * cxv;
  if (p == 2) {
    *c = 1.0 - 2.0 / 3.0 * s2;
    *ct = cxv * (5.0 + c2) / 6.0;
  } else {
    *c = 1.0 - s2 + 2.0 / 15.0 * s2 * s2;
    *ct = cxv * (c2 * c2 + 58.0 * c2 + 61.0) / 120.0;
  }
}

// Solid-harmonic form of y_l^m: with r the observer-relative node position,
// R = |r| and s = r_x + i r_y,  y_l^m(r / R) = Q_lm(r_z, R^2) s^m / R^l, where
// Q_lm = c_lm(u_z) R^(l-m) (c_lm: the z factor of ylm_one) written as
// z^odd (A z^4 + B z^2 R^2 + C R^4 + D z^2 + E R^2 + F) with z = r_z.
struct SolidQ {
  double A, B, C, D, E, F;
  int odd;
};

__device__ __forceinline__ SolidQ solid_coef(int l, int m) {
  SolidQ q = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0};
  switch (l * 8 + m) {
    case 0: q.F = 1.f; break;
    case 8: q.odd = 1; q.F = 1.f; break;
    case 9: q.F = -0.70710678118654752440; break;
    case 16: q.D = 1.5; q.E = -0.5; break;
    case 17: q.odd = 1; q.F = -1.22474487139158904910; break;
    case 18: q.F = 0.61237243569579452455; break;
    case 24: q.odd = 1; q.D = 2.5; q.E = -1.5; break;
    case 25: q.D = -2.16506350946109661690; q.E = 0.43301270189221932338; break;
    case 26: q.odd = 1; q.F = 1.36930639376291528364; break;
    case 27: q.F = -0.55901699437494742410; break;
    case 32: q.A = 4.375; q.B = -3.75; q.C = 0.375; break;
    case 33: q.odd = 1; q.D = -3.91311896062463196870; q.E = 1.67705098312484227230; break;
    case 34: q.D = 2.76699295264733191550; q.E = -0.39528470752104741650; break;
    case 35: q.odd = 1; q.F = -1.47901994577490951707; break;
    default: q.F = 0.52291251658379721749; break;  // l = 4, m = 4
  }
  return q;
}

template <typename T>
__device__ __forceinline__ T solid_eval(const SolidQ& q, T z, T r2) {
  const T z2 = z * z;
  const T v = (T(q.A) * z2 + T(q.B) * r2 + T(q.D)) * z2 + (T(q.C) * r2 + T(q.E)) * r2 + T(q.F);
  return q.odd ? v * z : v;
}

// Re (part 0) or Im (part 1) of (x + i y)^m
template <typename T>
__device__ __forceinline__ T cpow_part(T x, T y, int m, int part) {
  T sr = T(1), si = T(0);
  for (int k = 0; k < m; ++k) {
    const T t = sr * x - si * y;
    si = sr * y + si * x;
    sr = t;
  }
  return part ? si : sr;
}

}  // namespace cnpc
