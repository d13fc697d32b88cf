// Y_lm-weighted transforms, de-interlacing, F_l assembly and FP64 shell binning.
#include "spectra.h"

namespace cnpc {

// --------------------------------------------------------------- geometry --
struct Geo {
  double h;        // mesh spacing L / N
  double obs[3];   // observer (local line of sight)
  double los[3];   // fixed line of sight
  int global_los;
};

static Geo make_geo(const cnpc_mesh_desc* d) {
  Geo g;
  g.h = d->boxsize / d->n;
  for (int i = 0; i < 3; ++i) { g.obs[i] = d->observer[i]; g.los[i] = d->los[i]; }
  g.global_los = d->los_mode == CNPC_LOS_GLOBAL;
  return g;
}

struct FieldTable {
  int nf;
  signed char ell[32], m[32], part[32];
};

static int field_table(int nells, const int32_t* ells, FieldTable* ft) {
  int f = 0;
  for (int q = 0; q < nells; ++q) {
    const int l = ells[q];
    for (int m = 0; m <= l; ++m) {
      for (int p = 0; p < (m == 0 ? 1 : 2); ++p) {
        if (f >= 32) return -1;
        ft->ell[f] = (signed char)l;
        ft->m[f] = (signed char)m;
        ft->part[f] = (signed char)p;
        ++f;
      }
    }
  }
  ft->nf = f;
  return f;
}

template <typename T>
__device__ __forceinline__ void node_dir(const Geo& g, int ix, int iy, int iz, T* u) {
  if (g.global_los) {
    u[0] = T(g.los[0]); u[1] = T(g.los[1]); u[2] = T(g.los[2]);
    return;
  }
  const T rx = T(ix * g.h - g.obs[0]), ry = T(iy * g.h - g.obs[1]), rz = T(iz * g.h - g.obs[2]);
  const T inv = T(1) / sqrt(rx * rx + ry * ry + rz * rz);
  u[0] = rx * inv; u[1] = ry * inv; u[2] = rz * inv;
}

// ------------------------------------------------ materialised ylm fields --
template <typename T>
__global__ void __launch_bounds__(256) k_ylm_fields(const T* __restrict__ delta, T* __restrict__ out,
                                                    int n, int ell, Geo g) {
  const int64_t n3 = (int64_t)n * n * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int iz = (int)(i % n), iy = (int)((i / n) % n), ix = (int)(i / ((int64_t)n * n));
    T u[3];
    node_dir<T>(g, ix, iy, iz, u);
    T re[5], im[5];
    racah_ylm<T>(ell, u[0], u[1], u[2], re, im);
    const T dv = delta[i];
    out[i] = dv * re[0];
    for (int m = 1; m <= ell; ++m) {
      out[(2 * m - 1) * n3 + i] = dv * re[m];
      out[(2 * m) * n3 + i] = dv * im[m];
    }
  }
}

// ------------------------------------------ fused ylm prologue z-pass r2c --
// One row pair (ix, 2j), (ix, 2j+1) of delta per workgroup; fields [f0, f0+nfc)
// are formed in LDS and transformed; kz < kz_keep is written for each field.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_zpass_ylm(const T* __restrict__ delta, cx<T>* __restrict__ out,
                                                   FieldTable ft, int f0, int nfc, int kz_keep,
                                                   int64_t fstride, Geo g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* A = tw + N;
  cx<T>* B = A + nfc * N;
  load_twiddles<T, N, -1>(tw);
  const int q = blockIdx.x;
  const int ix = q / (N / 2), iy0 = 2 * (q - ix * (N / 2));
  const T* r0 = delta + ((int64_t)ix * N + iy0) * N;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    const T d0 = r0[e], d1 = r0[N + e];
    T u0[3], u1[3];
    node_dir<T>(g, ix, iy0, e, u0);
    node_dir<T>(g, ix, iy0 + 1, e, u1);
    int cur = -1;
    T re0[5], im0[5], re1[5], im1[5];
    for (int f = 0; f < nfc; ++f) {
      const int l = ft.ell[f0 + f], m = ft.m[f0 + f], p = ft.part[f0 + f];
      if (l != cur) {
        racah_ylm<T>(l, u0[0], u0[1], u0[2], re0, im0);
        racah_ylm<T>(l, u1[0], u1[1], u1[2], re1, im1);
        cur = l;
      }
      const T w0 = p ? im0[m] : re0[m];
      const T w1 = p ? im1[m] : re1[m];
      A[f * N + e] = cx<T>{d0 * w0, d1 * w1};
    }
  }
  __syncthreads();
  cx<T>* Z = fft_lds<T, N, -1, false>(A, B, nfc, 0, N, 1, tw);
  for (int idx = threadIdx.x; idx < nfc * kz_keep; idx += blockDim.x) {
    const int f = idx / kz_keep, k = idx - f * kz_keep;
    const cx<T> zk = Z[f * N + k];
    const cx<T> zm = cconj(Z[f * N + ((N - k) & (N - 1))]);
    const cx<T> a = cscale(cadd(zk, zm), T(0.5));
    const cx<T> dd = csub(zk, zm);
    const cx<T> b = {T(0.5) * dd.y, T(-0.5) * dd.x};
    cx<T>* o = out + (int64_t)(f0 + f) * fstride + ((int64_t)ix * N + iy0) * kz_keep;
    o[k] = a;
    o[kz_keep + k] = b;
  }
}

// One Racah-normalised harmonic component: Re (part 0) or Im (part 1) of
// y_l^m(u) for the unit vector u = (x, y, z) (same polynomials as racah_ylm).
template <typename T>
__device__ __forceinline__ T ylm_one(int l, int m, int part, T x, T y, T z) {
  T sr = T(1), si = T(0);  // (x + i y)^m
  for (int k = 0; k < m; ++k) {
    const T t = sr * x - si * y;
    si = sr * y + si * x;
    sr = t;
  }
  const T z2 = z * z;
  T c;
  switch (l * 8 + m) {
    case 0: c = T(1); break;
    case 8: c = z; break;
    case 9: c = T(-0.70710678118654752440); break;
    case 16: c = T(0.5) * (T(3) * z2 - T(1)); break;
    case 17: c = T(-1.22474487139158904910) * z; break;
    case 18: c = T(0.61237243569579452455); break;
    case 24: c = T(0.5) * z * (T(5) * z2 - T(3)); break;
    case 25: c = T(-0.43301270189221932338) * (T(5) * z2 - T(1)); break;
    case 26: c = T(1.36930639376291528364) * z; break;
    case 27: c = T(-0.55901699437494742410); break;
    case 32: c = T(0.125) * (T(35) * z2 * z2 - T(30) * z2 + T(3)); break;
    case 33: c = T(-0.55901699437494742410) * z * (T(7) * z2 - T(3)); break;
    case 34: c = T(0.39528470752104741650) * (T(7) * z2 - T(1)); break;
    case 35: c = T(-1.47901994577490951707) * z; break;
    default: c = T(0.52291251658379721749); break;  // l = 4, m = 4
  }
  return c * (part ? si : sr);
}

// R^-L for R^2 = q (FP32: hardware reciprocal / reciprocal square root).
template <typename T, int L>
__device__ __forceinline__ T inv_pow_r(T q) {
  if constexpr (L == 0) return T(1);
  T i2;
  if constexpr (sizeof(T) == 4) i2 = __builtin_amdgcn_rcpf(q);
  else i2 = T(1) / q;
  T r = (L & 2) ? i2 : T(1);
  if constexpr (L >= 4) r *= i2 * i2;
  if constexpr (L & 1) {
    if constexpr (sizeof(T) == 4) r *= __builtin_amdgcn_rsqf(q);
    else r /= sqrt(q);
  }
  return r;
}

// d0, d1 *= R^-K at the nodes z = rank + R n2 of the two rows (R^2 = rho + r_z^2)
template <typename T, int R, int K>
__device__ __forceinline__ void scale_rows(T* d0, T* d1, T rz0, T dz, T rho0, T rho1) {
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    T za = rz0 + T(n2) * dz;
    asm volatile("" : "+v"(za));
    d0[n2] *= inv_pow_r<T, K>(rho0 + za * za);
    d1[n2] *= inv_pow_r<T, K>(rho1 + za * za);
  }
}

// Q_lm(z, rho^2 + z^2) s = (c4 z^2 + c2) z^2 + c0, times z when Q_lm is odd:
// the solid-harmonic polynomial along one row (rho^2 = r_x^2 + r_y^2), with
// the row factor s = Re / Im (r_x + i r_y)^m folded in.
template <typename T>
struct ZPoly {
  T c4, c2, c0;
};

template <typename T>
__device__ __forceinline__ ZPoly<T> zpoly(const SolidQ& q, T rho2, T s) {
  // Q = (A z^2 + B R^2 + D) z^2 + (C R^2 + E) R^2 + F with R^2 = rho^2 + z^2
  const T r = rho2;
  ZPoly<T> c;
  c.c4 = T(q.A + q.B + q.C) * s;
  c.c2 = (T(q.B + 2.0 * q.C) * r + T(q.D + q.E)) * s;
  c.c0 = ((T(q.C) * r + T(q.E)) * r + T(q.F)) * s;
  return c;
}

// v[n2] = (d0 w(row 0), d1 w(row 1)) at the nodes z = rank + R n2, with
// w = Q_lm s along each row and d = delta R^-l
template <typename T, int R, bool ODD>
__device__ __forceinline__ void weigh_z(cx<T>* v, const T* d0, const T* d1, T rz0, T dz, const ZPoly<T>& a,
                                       const ZPoly<T>& b) {
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    // opaque copy: keeps r_z and r_z^2 of all nodes from being hoisted out of
    // the field loop into registers
    T za = rz0 + T(n2) * dz;
    asm volatile("" : "+v"(za));
    const T z2 = za * za;
    T w0 = (a.c4 * z2 + a.c2) * z2 + a.c0;
    T w1 = (b.c4 * z2 + b.c2) * z2 + b.c0;
    if constexpr (ODD) {
      w0 *= za;
      w1 *= za;
    }
    v[n2] = cx<T>{d0[n2] * w0, d1[n2] * w1};
  }
}

// Register z-pass for N = R^2: a group of R lanes owns one row pair (ix, 2j),
// (ix, 2j+1) of delta and, field after field, forms the weighted pair as one
// complex row, transforms it with row_fft_rr and writes kz < kz_keep of both
// real rows (two-for-one split).  Local line of sight: the weight of a node is
// Q_lm(r_z, R^2) R^-l times the row constant Re / Im (r_x + i r_y)^m.
template <typename T, int R>
__global__ void __launch_bounds__(256, 3) k_zpass_ylm_rr(const T* __restrict__ delta, cx<T>* __restrict__ out,
                                                      FieldTable ft, int kz_keep, int64_t fstride, Geo g) {
  constexpr int N = R * R;
  constexpr int GR = 256 / R;  // row pairs per workgroup
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T, N, -1>(tw);
  const int grp = threadIdx.x / R, rank = threadIdx.x % R;
  cx<T>* buf = tw + N + grp * (R * (R + 1));
  const int q = blockIdx.x * GR + grp;
  const int ix = q / (N / 2), iy0 = 2 * (q - ix * (N / 2));
  const T* r0 = delta + ((int64_t)ix * N + iy0) * N;
  // delta R^-pw of the two rows; pw follows the l of the current field run
  // (local line of sight), from delta itself whenever l drops
  T d0[R], d1[R];
  int pw = 0;
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int z = rank + R * n2;
    d0[n2] = r0[z];
    d1[n2] = r0[N + z];
  }
  // r_z of node z = rank + R n2 is rz0 + n2 dz (recomputed where needed)
  const T rz0 = T(rank * g.h - g.obs[2]), dz = T(R * g.h);
  const T rx = T(ix * g.h - g.obs[0]);
  const T ry0 = T(iy0 * g.h - g.obs[1]), ry1 = T((iy0 + 1) * g.h - g.obs[1]);
  const T rho0 = rx * rx + ry0 * ry0, rho1 = rx * rx + ry1 * ry1;
  __syncthreads();
  const int src = (R - rank) & (R - 1);
  const int K2 = (kz_keep + R - 1) / R;
  cx<T>* orow = out + ((int64_t)ix * N + iy0) * kz_keep;
  for (int f0 = 0; f0 < ft.nf;) {
    const int l = ft.ell[f0];
    int f1 = f0 + 1;
    while (f1 < ft.nf && ft.ell[f1] == l) ++f1;
    if (!g.global_los && l != pw) {
      if (l < pw) {
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) {
          const int z = rank + R * n2;
          d0[n2] = r0[z];
          d1[n2] = r0[N + z];
        }
        pw = 0;
      }
      switch (l - pw) {
        case 1: scale_rows<T, R, 1>(d0, d1, rz0, dz, rho0, rho1); break;
        case 2: scale_rows<T, R, 2>(d0, d1, rz0, dz, rho0, rho1); break;
        case 3: scale_rows<T, R, 3>(d0, d1, rz0, dz, rho0, rho1); break;
        case 4: scale_rows<T, R, 4>(d0, d1, rz0, dz, rho0, rho1); break;
        default: break;
      }
      pw = l;
    }
    for (int f = f0; f < f1; ++f) {
      const int m = ft.m[f], p = ft.part[f];
      cx<T> v[R];
      if (g.global_los) {
        const T w = ylm_one<T>(l, m, p, T(g.los[0]), T(g.los[1]), T(g.los[2]));
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) v[n2] = cx<T>{d0[n2] * w, d1[n2] * w};
      } else {
        const T s0 = cpow_part<T>(rx, ry0, m, p), s1 = cpow_part<T>(rx, ry1, m, p);
        const SolidQ qc = solid_coef(l, m);
        const ZPoly<T> a = zpoly<T>(qc, rho0, s0), b = zpoly<T>(qc, rho1, s1);
        if (qc.odd) weigh_z<T, R, true>(v, d0, d1, rz0, dz, a, b);
        else weigh_z<T, R, false>(v, d0, d1, rz0, dz, a, b);
      }
      row_fft_rr<T, R, -1>(v, rank, buf, tw);
      // lane k1 holds Z[k1 + R k2]; Z[N - k] sits in lane (R - k1) & (R - 1),
      // register R - 1 - k2 (k1 > 0) or in this lane, register (R - k2) & (R - 1)
      cx<T>* o = orow + (int64_t)f * fstride;
#pragma unroll
      for (int k2 = 0; k2 < R / 2; ++k2) {
        if (k2 < K2) {
          const cx<T> a = v[R - 1 - k2];
          const cx<T> sh = {__shfl(a.x, src, R), __shfl(a.y, src, R)};
          const cx<T> zm = cconj(rank ? sh : v[(R - k2) & (R - 1)]);
          const cx<T> zk = v[k2];
          const int k = rank + R * k2;
          if (k < kz_keep) {
            const cx<T> dd = csub(zk, zm);
            o[k] = cscale(cadd(zk, zm), T(0.5));
            o[kz_keep + k] = cx<T>{T(0.5) * dd.y, T(-0.5) * dd.x};
          }
        }
      }
    }
    f0 = f1;
  }
}

// r_z^J for a compile-time power J
template <typename T, int J>
__device__ __forceinline__ T zpow(T z) {
  if constexpr (J == 0) return T(1);
  else if constexpr (J == 1) return z;
  else if constexpr (J == 2) return z * z;
  else if constexpr (J == 3) return z * z * z;
  else { const T z2 = z * z; return z2 * z2; }
}

// basis J of the row pair: transform of (d0, d1) r_z^J, split per row at the
// kept kz = rank + R k2 (k2 < K2M): row 0 into g0[k2], row 1 into g1[k2]
template <typename T, int R, int K2M, int J>
__device__ __forceinline__ void zbasis(const T* d0, const T* d1, T rz0, T dz, int rank, int src, cx<T>* buf,
                                       const cx<T>* tw, cx<T>* g0, cx<T>* g1) {
  cx<T> v[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    T za = rz0 + T(n2) * dz;
    asm volatile("" : "+v"(za));
    const T w = zpow<T, J>(za);
    v[n2] = J == 0 ? cx<T>{d0[n2], d1[n2]} : cx<T>{d0[n2] * w, d1[n2] * w};
  }
  // an opaque lane index per call: keeps the twiddle reads of the bases from
  // being merged into one register copy held across all of them
  int lane = rank;
  asm volatile("" : "+v"(lane));
  row_fft_rr<T, R, -1, true>(v, lane, buf, tw);
  // lane k1 holds Z[k1 + R k2]; Z[N - k] sits in lane (R - k1) & (R - 1),
  // register R - 1 - k2 (k1 > 0) or in this lane, register (R - k2) & (R - 1)
#pragma unroll
  for (int k2 = 0; k2 < K2M; ++k2) {
    const cx<T> a = v[R - 1 - k2];
    const cx<T> sh = {__shfl(a.x, src, R), __shfl(a.y, src, R)};
    const cx<T> zm = cconj(rank ? sh : v[(R - k2) & (R - 1)]);
    const cx<T> zk = v[k2];
    const cx<T> dd = csub(zk, zm);
    g0[k2] = cscale(cadd(zk, zm), T(0.5));
    g1[k2] = cx<T>{T(0.5) * dd.y, T(-0.5) * dd.x};
  }
}

// c0 g[b0] + c2 g[b0 + 2] + c4 g[b0 + 4] at one kz (bases past 4 have c = 0)
template <typename T, int K2M, int B0>
__device__ __forceinline__ cx<T> zcombine(const cx<T> (*g)[K2M], int k2, T c0, T c2, T c4) {
  cx<T> r = cscale(g[B0][k2], c0);
  r = cx<T>{r.x + c2 * g[B0 + 2][k2].x, r.y + c2 * g[B0 + 2][k2].y};
  if constexpr (B0 + 4 <= 4) r = cx<T>{r.x + c4 * g[B0 + 4][k2].x, r.y + c4 * g[B0 + 4][k2].y};
  return r;
}

// Register z-pass by powers of r_z (N = R^2, l <= 4, kz_keep <= K2M R).  With
// R^2 = rho^2 + r_z^2 (rho^2 = r_x^2 + r_y^2, fixed along a z row), the
// weight y_l^m = Q_lm(r_z, R^2) s^m / R^l of a field is, over the common
// R^-L of its parity class (L the largest l of that parity in the table),
// the row constant times the polynomial Q_lm R^(L - l) in r_z of degree
// L - m <= 4 (R^(L - l) = (rho^2 + r_z^2)^((L - l) / 2) for even L - l).  The
// transform is linear, so every field's row spectrum is sum_j e_j G_j with G_j
// the spectrum of delta R^-L r_z^j, j = 0..L: L + 1 transforms per parity
// class (two rows as one complex sequence, split per row at the kept kz) in
// place of 2l + 1 per l, e.g. 5 for l = 2, 4 against 14; one transform for all
// fields with a global line of sight (G_0 of delta itself).  Same outputs as
// k_zpass_ylm_rr up to rounding.
template <typename T, int R, int K2M>
__global__ void __launch_bounds__(256, K2M == 2 ? 3 : 2) k_zpass_ylm_basis(const T* __restrict__ delta, cx<T>* __restrict__ out,
                                                         FieldTable ft, int kz_keep, int64_t fstride, Geo g) {
  constexpr int N = R * R;
  constexpr int GR = 256 / R;  // row pairs per workgroup
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T, N, -1>(tw);
  const int grp = threadIdx.x / R, rank = threadIdx.x % R;
  cx<T>* buf = tw + N + grp * (R * (R + 1));
  const int q = blockIdx.x * GR + grp;
  const int ix = q / (N / 2), iy0 = 2 * (q - ix * (N / 2));
  const T* r0 = delta + ((int64_t)ix * N + iy0) * N;
  T d0[R], d1[R];
  int pw = 0;
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int z = rank + R * n2;
    d0[n2] = r0[z];
    d1[n2] = r0[N + z];
  }
  const T rz0 = T(rank * g.h - g.obs[2]), dz = T(R * g.h);
  const T rx = T(ix * g.h - g.obs[0]);
  const T ry0 = T(iy0 * g.h - g.obs[1]), ry1 = T((iy0 + 1) * g.h - g.obs[1]);
  const T rho0 = rx * rx + ry0 * ry0, rho1 = rx * rx + ry1 * ry1;
  __syncthreads();  // twiddles
  const int src = (R - rank) & (R - 1);
  cx<T>* orow = out + ((int64_t)ix * N + iy0) * kz_keep;
  cx<T> g0[5][K2M], g1[5][K2M];
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int k2 = 0; k2 < K2M; ++k2) g0[j][k2] = g1[j][k2] = cx<T>{T(0), T(0)};
  bool have = false;  // a global line of sight needs G_0 once
  for (int par = 1; par >= 0; --par) {  // odd l, then even l
    int L = -1;
    for (int f = 0; f < ft.nf; ++f)
      if ((ft.ell[f] & 1) == par && ft.ell[f] > L) L = ft.ell[f];
    if (L < 0) continue;
    if (!g.global_los) {
      if (L != pw) {
        if (L < pw) {
#pragma unroll
          for (int n2 = 0; n2 < R; ++n2) {
            const int z = rank + R * n2;
            d0[n2] = r0[z];
            d1[n2] = r0[N + z];
          }
          pw = 0;
        }
        switch (L - pw) {
          case 1: scale_rows<T, R, 1>(d0, d1, rz0, dz, rho0, rho1); break;
          case 2: scale_rows<T, R, 2>(d0, d1, rz0, dz, rho0, rho1); break;
          case 3: scale_rows<T, R, 3>(d0, d1, rz0, dz, rho0, rho1); break;
          case 4: scale_rows<T, R, 4>(d0, d1, rz0, dz, rho0, rho1); break;
          default: break;
        }
        pw = L;
      }
      zbasis<T, R, K2M, 0>(d0, d1, rz0, dz, rank, src, buf, tw, g0[0], g1[0]);
      if (L >= 1) zbasis<T, R, K2M, 1>(d0, d1, rz0, dz, rank, src, buf, tw, g0[1], g1[1]);
      if (L >= 2) zbasis<T, R, K2M, 2>(d0, d1, rz0, dz, rank, src, buf, tw, g0[2], g1[2]);
      if (L >= 3) zbasis<T, R, K2M, 3>(d0, d1, rz0, dz, rank, src, buf, tw, g0[3], g1[3]);
      if (L >= 4) zbasis<T, R, K2M, 4>(d0, d1, rz0, dz, rank, src, buf, tw, g0[4], g1[4]);
    } else if (!have) {
      zbasis<T, R, K2M, 0>(d0, d1, rz0, dz, rank, src, buf, tw, g0[0], g1[0]);
      have = true;
    }
    for (int f = 0; f < ft.nf; ++f) {
      const int l = ft.ell[f];
      if ((l & 1) != par) continue;
      const int m = ft.m[f], p = ft.part[f];
      // coefficients of r_z^(odd + 2i), i = 0..2, for row 0 (a) and row 1 (b)
      T a0, a2, a4, b0, b2, b4;
      bool odd = false;
      if (g.global_los) {
        a0 = b0 = ylm_one<T>(l, m, p, T(g.los[0]), T(g.los[1]), T(g.los[2]));
        a2 = a4 = b2 = b4 = T(0);
      } else {
        const T s0 = cpow_part<T>(rx, ry0, m, p), s1 = cpow_part<T>(rx, ry1, m, p);
        const SolidQ qc = solid_coef(l, m);
        const ZPoly<T> a = zpoly<T>(qc, rho0, s0), b = zpoly<T>(qc, rho1, s1);
        odd = qc.odd != 0;
        a0 = a.c0; a2 = a.c2; a4 = a.c4;
        b0 = b.c0; b2 = b.c2; b4 = b.c4;
        for (int k = l; k < L; k += 2) {  // times rho^2 + r_z^2 (the degree stays <= 4)
          a4 = a4 * rho0 + a2; a2 = a2 * rho0 + a0; a0 = a0 * rho0;
          b4 = b4 * rho1 + b2; b2 = b2 * rho1 + b0; b0 = b0 * rho1;
        }
      }
      cx<T>* o = orow + (int64_t)f * fstride;
#pragma unroll
      for (int k2 = 0; k2 < K2M; ++k2) {
        const int k = rank + R * k2;
        if (k < kz_keep) {
          if (odd) {
            o[k] = zcombine<T, K2M, 1>(g0, k2, a0, a2, a4);
            o[kz_keep + k] = zcombine<T, K2M, 1>(g1, k2, b0, b2, b4);
          } else {
            o[k] = zcombine<T, K2M, 0>(g0, k2, a0, a2, a4);
            o[kz_keep + k] = zcombine<T, K2M, 0>(g1, k2, b0, b2, b4);
          }
        }
      }
    }
  }
}

// ---------------------------------- z-power bases combined in the y pass --
// Bases of a field table: per parity class of l (odd first) the spectra of
// delta R^-L r_z^j, j = 0..L (L the class's largest l), at basis indices
// off[c] + j; a global line of sight has the one basis delta.  Field f is
// sum_i e_i B[bo[f] + 2 i] over i < nt[f] (bo = class offset + parity of
// l - m, nt = 1 + (L - m - that parity) / 2).
struct YlmBases {
  int nclass, nb;
  int L[2], off[2];
  signed char bo[32], nt[32];
};

static YlmBases ylm_bases(const FieldTable& ft, bool global_los) {
  YlmBases yb{};
  int Lp[2] = {-1, -1};  // by parity of l
  for (int f = 0; f < ft.nf; ++f) Lp[ft.ell[f] & 1] = std::max(Lp[ft.ell[f] & 1], (int)ft.ell[f]);
  if (global_los) {
    yb.nclass = 1;
    yb.L[0] = 0;
    yb.off[0] = 0;
    yb.nb = 1;
    for (int f = 0; f < ft.nf; ++f) { yb.bo[f] = 0; yb.nt[f] = 1; }
    return yb;
  }
  int off[2] = {0, 0}, nb = 0;
  // classes by ascending L, so that the R^-L scaling of delta only grows
  const int first = Lp[1] >= 0 && (Lp[0] < 0 || Lp[1] < Lp[0]) ? 1 : 0;
  for (int par : {first, 1 - first}) {
    if (Lp[par] < 0) continue;
    yb.L[yb.nclass] = Lp[par];
    yb.off[yb.nclass] = nb;
    off[par] = nb;
    nb += Lp[par] + 1;
    ++yb.nclass;
  }
  yb.nb = nb;
  for (int f = 0; f < ft.nf; ++f) {
    const int l = ft.ell[f], m = ft.m[f], odd = (l - m) & 1, L = Lp[l & 1];
    yb.bo[f] = (signed char)(off[l & 1] + odd);
    yb.nt[f] = (signed char)(1 + (L - m - odd) / 2);
  }
  return yb;
}

// Coefficients e_0, e_2, e_4 of the fields' polynomials in r_z on every z row:
// coef[f][ix][iy] = (e_0, e_2, e_4, 0), the row constant of y_l^m times
// Q_lm R^(L - l) (ZPoly times (rho^2 + r_z^2)^((L - l) / 2)); the weight
// itself for a global line of sight.
template <typename T>
__global__ void __launch_bounds__(256) k_ylm_coef(FieldTable ft, YlmBases yb, int n, Geo g, T* __restrict__ coef) {
  const int64_t nn = (int64_t)n * n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ft.nf * nn) return;
  const int f = (int)(i / nn);
  const int ix = (int)((i - f * nn) / n), iy = (int)(i % n);
  const int l = ft.ell[f], m = ft.m[f], p = ft.part[f];
  T e0, e2 = T(0), e4 = T(0);
  if (g.global_los) {
    e0 = ylm_one<T>(l, m, p, T(g.los[0]), T(g.los[1]), T(g.los[2]));
  } else {
    const T rx = T(ix * g.h - g.obs[0]), ry = T(iy * g.h - g.obs[1]);
    const T rho = rx * rx + ry * ry;
    const ZPoly<T> a = zpoly<T>(solid_coef(l, m), rho, cpow_part<T>(rx, ry, m, p));
    e0 = a.c0;
    e2 = a.c2;
    e4 = a.c4;
    const int L = yb.L[0] % 2 == l % 2 ? yb.L[0] : yb.L[1];
    for (int k = l; k < L; k += 2) {  // times rho^2 + r_z^2 (the degree stays <= 4)
      e4 = e4 * rho + e2;
      e2 = e2 * rho + e0;
      e0 = e0 * rho;
    }
  }
  T* o = coef + 4 * i;
  o[0] = e0;
  o[1] = e2;
  o[2] = e4;
  o[3] = T(0);
}

// Register z pass of the bases alone (N = R^2): per row pair the spectra of
// delta R^-L r_z^j (both rows as one complex sequence, split per row) at
// kz < kz_keep, written as planes [basis][x][y][kz] (layout of the fields of
// k_zpass_ylm_rr).  ZIN = false: delta is the real mesh; ZIN = true: delta is
// given as its z half spectra (rows of N/2 complex values, kz < N/2, Nyquist
// zero; the layout k_zpass_c2r_rr takes), inverse-transformed here first, so
// that the real mesh is never stored (the classes then have ascending L and
// delta is never re-read).
template <typename T, int R, bool ZIN>
__global__ void __launch_bounds__(256, 3) k_zpass_ylm_bases(const void* __restrict__ delta_in,
                                                         cx<T>* __restrict__ out, YlmBases yb, int kz_keep,
                                                         int64_t bstride, Geo g) {
  constexpr int N = R * R, H = N / 2;
  constexpr int GR = 256 / R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twi = tw + N;  // inverse twiddles (ZIN)
  load_twiddles<T, N, -1>(tw);
  if constexpr (ZIN) load_twiddles<T, N, 1>(twi);
  const int grp = threadIdx.x / R, rank = threadIdx.x % R;
  cx<T>* buf = tw + (ZIN ? 2 : 1) * N + grp * (R * (R + 1));
  const int q = blockIdx.x * GR + grp;
  const int ix = q / (N / 2), iy0 = 2 * (q - ix * (N / 2));
  const T* r0 = reinterpret_cast<const T*>(delta_in) + ((int64_t)ix * N + iy0) * N;
  T d0[R], d1[R];
  int pw = 0;
  if constexpr (ZIN) {
    // both rows as one complex sequence A + i B from their half spectra A, B
    // (clamped straight-line loads; k = N/2 is the zero Nyquist term)
    const cx<T>* z0 = reinterpret_cast<const cx<T>*>(delta_in) + (int64_t)2 * q * H;
    cx<T> v[R];
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
      const int k = rank + R * n2;
      const int kk = k < H ? k : N - k;  // <= H
      const int kc = kk < H ? kk : H - 1;
      const cx<T> a = z0[kc], b = z0[H + kc];
      cx<T> zv = k < H ? cx<T>{a.x - b.y, a.y + b.x} : cx<T>{a.x + b.y, b.x - a.y};
      v[n2] = kk < H ? zv : cx<T>{T(0), T(0)};
    }
    __syncthreads();  // twiddles
    row_fft_rr<T, R, 1, true>(v, rank, buf, twi);
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
      d0[n2] = v[n2].x;
      d1[n2] = v[n2].y;
    }
  } else {
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) {
      const int z = rank + R * n2;
      d0[n2] = r0[z];
      d1[n2] = r0[N + z];
    }
  }
  const T rz0 = T(rank * g.h - g.obs[2]), dz = T(R * g.h);
  const T rx = T(ix * g.h - g.obs[0]);
  const T ry0 = T(iy0 * g.h - g.obs[1]), ry1 = T((iy0 + 1) * g.h - g.obs[1]);
  const T rho0 = rx * rx + ry0 * ry0, rho1 = rx * rx + ry1 * ry1;
  __syncthreads();  // twiddles
  const int src = (R - rank) & (R - 1);
  const int K2 = (kz_keep + R - 1) / R;
  cx<T>* orow = out + ((int64_t)ix * N + iy0) * kz_keep;
  for (int cl = 0; cl < yb.nclass; ++cl) {
    const int L = yb.L[cl];
    if (!g.global_los && L != pw) {
      if (!ZIN && L < pw) {
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) {
          const int z = rank + R * n2;
          d0[n2] = r0[z];
          d1[n2] = r0[N + z];
        }
        pw = 0;
      }
      switch (L - pw) {
        case 1: scale_rows<T, R, 1>(d0, d1, rz0, dz, rho0, rho1); break;
        case 2: scale_rows<T, R, 2>(d0, d1, rz0, dz, rho0, rho1); break;
        case 3: scale_rows<T, R, 3>(d0, d1, rz0, dz, rho0, rho1); break;
        case 4: scale_rows<T, R, 4>(d0, d1, rz0, dz, rho0, rho1); break;
        default: break;
      }
      pw = L;
    }
#pragma unroll
    for (int j = 0; j <= 4; ++j) {
      if (j > L) break;
      cx<T> v[R];
#pragma unroll
      for (int n2 = 0; n2 < R; ++n2) {
        T za = rz0 + T(n2) * dz;
        asm volatile("" : "+v"(za));
        T w = T(1);
#pragma unroll
        for (int e = 0; e < j; ++e) w *= za;
        v[n2] = cx<T>{d0[n2] * w, d1[n2] * w};
      }
      row_fft_rr<T, R, -1, true>(v, rank, buf, tw);
      cx<T>* o = orow + (int64_t)(yb.off[cl] + j) * bstride;
#pragma unroll
      for (int k2 = 0; k2 < R / 2; ++k2) {
        if (k2 < K2) {
          const cx<T> a = v[R - 1 - k2];
          const cx<T> sh = {__shfl(a.x, src, R), __shfl(a.y, src, R)};
          const cx<T> zm = cconj(rank ? sh : v[(R - k2) & (R - 1)]);
          const cx<T> zk = v[k2];
          const int k = rank + R * k2;
          if (k < kz_keep) {
            const cx<T> dd = csub(zk, zm);
            o[k] = cscale(cadd(zk, zm), T(0.5));
            o[kz_keep + k] = cx<T>{T(0.5) * dd.y, T(-0.5) * dd.x};
          }
        }
      }
    }
  }
}

// rows rank + R n2 of column kz of a field with NT terms: sum_i e_i B[bo + 2i]
// (bases from global memory, all loads issued before the first use;
// coefficients e from the workgroup's copy in LDS)
template <typename T, int R, int NT>
__device__ __forceinline__ void ylm_combine(cx<T>* v, const cx<T>* __restrict__ b0, const T* ecf, int rank,
                                            int64_t bstride, int m) {
  cx<T> u[NT][R];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int n2 = 0; n2 < R; ++n2) u[i][n2] = b0[(int64_t)(2 * i) * bstride + (int64_t)(rank + R * n2) * m];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const T* e = ecf + 4 * (rank + R * n2);
    cx<T> a = cscale(u[0][n2], e[0]);
#pragma unroll
    for (int i = 1; i < NT; ++i) a = cx<T>{a.x + e[i] * u[i][n2].x, a.y + e[i] * u[i][n2].y};
    v[n2] = a;
  }
}

// Forward y pass of the band z spectra of the Y_lm fields formed from the
// bases (N = R^2, W = 256 / R kz columns per workgroup): workgroup (ix, f, tile)
// reads at each of its rows y and columns kz the bases of field f, combines
// them with coef[f][ix][y], transforms along y and writes the band rows
// ky = -(m-1) .. m-1 (n = -m as zero) of plane (f, ix), layout [f][x][2m][m].
// Workgroups of one x plane run on one XCD (workgroup index mod 8 picks the
// XCD), so the fields of a plane read its bases from that XCD's L2.
template <typename T, int R>
__global__ void __launch_bounds__(256) k_colpass_ylm_rr(const cx<T>* __restrict__ bases, const T* __restrict__ coef,
                                                     cx<T>* __restrict__ out, YlmBases yb, int nf, int m) {
  constexpr int N = R * R, W = 256 / R, LOGW = (W == 8 ? 3 : W == 16 ? 4 : W == 32 ? 5 : 6);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* buf = tw + N;
  T* ecf = reinterpret_cast<T*>(buf + (size_t)N * W + 16 * R);  // [N][4] coefficients of the plane
  load_twiddles<T, N, -1>(tw);
  const int c = threadIdx.x & (W - 1), rank = threadIdx.x >> LOGW;
  const int tiles = m / W;
  const unsigned per = gridDim.x / 8;  // gridDim.x is a multiple of 8
  const unsigned lb = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  const int t = (int)(lb % (unsigned)tiles);
  const int pf = (int)(lb / (unsigned)tiles);
  const int ix = pf / nf, f = pf - ix * nf;
  const int kz = t * W + c;
  const int bo = yb.bo[f], nt = yb.nt[f];
  const int64_t bstride = (int64_t)N * N * m;
  const cx<T>* b0 = bases + (int64_t)bo * bstride + (int64_t)ix * N * m + kz;
  const T* cf = coef + (((int64_t)f * N + ix) * N) * 4;
  for (int i = threadIdx.x; i < N; i += 256)
    reinterpret_cast<float4*>(ecf)[i] = reinterpret_cast<const float4*>(cf)[i];  // T = float
  __syncthreads();  // twiddles, coefficients
  cx<T> v[R];
  if (nt == 1) ylm_combine<T, R, 1>(v, b0, ecf, rank, bstride, m);
  else if (nt == 2) ylm_combine<T, R, 2>(v, b0, ecf, rank, bstride, m);
  else ylm_combine<T, R, 3>(v, b0, ecf, rank, bstride, m);
  col_fft_rr<T, R, -1>(v, c, rank, buf, tw);
  cx<T>* dst = out + ((int64_t)f * N + ix) * 2 * m * m + kz;
#pragma unroll
  for (int k2 = 0; k2 < R; ++k2) {
    const int r = rank + R * k2;
    int j;
    if (r < m) j = r;
    else if (r >= N - m) j = r - N + 2 * m;
    else continue;
    dst[(int64_t)j * m] = v[k2];
  }
}

template <typename T, int R>
static cnpc_status zylm_rr(const T* delta, cx<T>* out, const FieldTable& ft, int kz, int64_t fstride,
                           const Geo& g, hipStream_t s) {
  constexpr int N = R * R, GR = 256 / R;
  const size_t lds = sizeof(cx<T>) * (N + (size_t)GR * R * (R + 1));
  const dim3 grid(N * (N / 2) / GR);
  // FP32 with kz_keep <= 4 R: powers of r_z (CNPC_TUNE_YLM_BASIS 1: one
  // transform per field); FP64 and wider bands: one transform per field
  const bool basis = kz <= 4 * R && tune_value(CNPC_TUNE_YLM_BASIS) != 1;
  kt_begin(CNPC_KT_ZR2C, s);
  if constexpr (sizeof(T) == 4) {
    if (basis && kz <= 2 * R)
      hipLaunchKernelGGL((k_zpass_ylm_basis<T, R, 2>), grid, dim3(256), lds, s, delta, out, ft, kz, fstride, g);
    else if (basis)
      hipLaunchKernelGGL((k_zpass_ylm_basis<T, R, 4>), grid, dim3(256), lds, s, delta, out, ft, kz, fstride, g);
    else
      hipLaunchKernelGGL((k_zpass_ylm_rr<T, R>), grid, dim3(256), lds, s, delta, out, ft, kz, fstride, g);
  } else {
    (void)basis;
    hipLaunchKernelGGL((k_zpass_ylm_rr<T, R>), grid, dim3(256), lds, s, delta, out, ft, kz, fstride, g);
  }
  kt_end(CNPC_KT_ZR2C, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

template <typename T, int N>
static cnpc_status zylm_n(const T* delta, cx<T>* out, const FieldTable& ft, int kz,
                          int64_t fstride, const Geo& g, hipStream_t s) {
  // fields per launch: two ping-pong buffers of nfc * N elements within the LDS limit
  const size_t per = 2 * N * sizeof(cx<T>);
  int nfc = (int)((lds_limit() - N * sizeof(cx<T>)) / per);
  if (nfc < 1) nfc = 1;
  if (nfc > ft.nf) nfc = ft.nf;
  for (int f0 = 0; f0 < ft.nf; f0 += nfc) {
    const int c = std::min(nfc, ft.nf - f0);
    const size_t lds = sizeof(cx<T>) * (N + 2 * c * N);
    kt_begin(CNPC_KT_ZR2C, s);
    hipLaunchKernelGGL((k_zpass_ylm<T, N>), dim3(N * (N / 2)), dim3(256), lds, s, delta, out, ft, f0, c,
                       kz, fstride, g);
    kt_end(CNPC_KT_ZR2C, s);
    CNPC_HIP(hipGetLastError());
  }
  return CNPC_OK;
}

template <typename T>
static cnpc_status zpass_ylm(int n, const T* delta, cx<T>* out, const FieldTable& ft, int kz,
                             int64_t fstride, const Geo& g, hipStream_t s) {
  switch (n) {
    case 16: return zylm_rr<T, 4>(delta, out, ft, kz, fstride, g, s);
    case 32: return zylm_n<T, 32>(delta, out, ft, kz, fstride, g, s);
    case 64:
      if (fft_register_passes()) return zylm_rr<T, 8>(delta, out, ft, kz, fstride, g, s);
      return zylm_n<T, 64>(delta, out, ft, kz, fstride, g, s);
    case 128: return zylm_n<T, 128>(delta, out, ft, kz, fstride, g, s);
    case 256:
      if (fft_register_passes()) return zylm_rr<T, 16>(delta, out, ft, kz, fstride, g, s);
      return zylm_n<T, 256>(delta, out, ft, kz, fstride, g, s);
    case 512: return zylm_n<T, 512>(delta, out, ft, kz, fstride, g, s);
    case 1024: return zylm_n<T, 1024>(delta, out, ft, kz, fstride, g, s);
    default: set_error("unsupported mesh size %d", n); return CNPC_EUNSUPPORTED;
  }
}

// y then x column passes of a band-pruned forward transform:
// w1 [batch][n][n][m] -> w2 [batch][n][2m][m] -> out [batch][2m][2m][m]
template <typename T>
cnpc_status band_forward_yx(int n, int dt, int batch, int m, const cx<T>* w1, cx<T>* w2, cx<T>* out,
                            hipStream_t s) {
  ColArgs ay = make_col(n, dt, (int64_t)n * m, (int64_t)2 * m * m, m, m, m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, w1, w2, ay, (int64_t)batch * n, s));
  ColArgs ax = make_col(n, dt, (int64_t)n * 2 * m * m, (int64_t)4 * m * m * m, (int64_t)2 * m * m,
                        (int64_t)2 * m * m, 2 * m * m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, w2, out, ax, batch, s));
  return CNPC_OK;
}
template cnpc_status band_forward_yx<float>(int, int, int, int, const cx<float>*, cx<float>*,
                                            cx<float>*, hipStream_t);
template cnpc_status band_forward_yx<double>(int, int, int, int, const cx<double>*, cx<double>*,
                                             cx<double>*, hipStream_t);

// FP32 at N = 256 with register passes, a band of whole 16-column tiles and
// CNPC_TUNE_YLM_BASIS 0: the z pass writes the z-power bases, the y pass forms
// the fields from them (coefficient table next to the bases in w1)
template <typename T>
static bool ylm_bases_route(int n, int m, const FieldTable& ft, const YlmBases& yb) {
  if (sizeof(T) != 4 || n != 256 || m % 16 != 0 || !fft_register_passes()) return false;
  if (tune_value(CNPC_TUNE_YLM_BASIS) == 1) return false;
  const size_t nn = (size_t)n * n;
  return yb.nb * nn * m * sizeof(cx<T>) + ft.nf * nn * 4 * sizeof(T) <= ft.nf * nn * m * sizeof(cx<T>);
}

// zspec: delta holds the z half spectra of the real mesh (bases route only)
template <typename T>
static cnpc_status ylm_r2c_t(const cnpc_mesh_desc* d, int band, const FieldTable& ft,
                             const T* delta, cx<T>* out, cx<T>* ws, const T* coef_in, bool zspec, hipStream_t s) {
  CNPC_TRY(ensure_twiddles());
  const int n = d->n, m = band;
  const int64_t nn = (int64_t)n * n;
  cx<T>* w1 = ws;
  cx<T>* w2 = ws + (int64_t)ft.nf * nn * m;
  const Geo g = make_geo(d);
  const YlmBases yb = ylm_bases(ft, g.global_los != 0);
  if constexpr (sizeof(T) == 4) {
    if (ylm_bases_route<T>(n, m, ft, yb)) {
      constexpr int R = 16, N = 256, GR = 256 / R;
      const T* coef = coef_in;
      kt_begin(CNPC_KT_ZR2C, s);
      if (!coef) {
        T* c = reinterpret_cast<T*>(w1 + (int64_t)yb.nb * nn * m);
        const int64_t ncoef = ft.nf * nn;
        hipLaunchKernelGGL((k_ylm_coef<T>), dim3((unsigned)((ncoef + 255) / 256)), dim3(256), 0, s, ft, yb, n, g, c);
        coef = c;
      }
      const size_t zlds = sizeof(cx<T>) * ((zspec ? 2 : 1) * N + (size_t)GR * R * (R + 1));
      if (zspec)
        hipLaunchKernelGGL((k_zpass_ylm_bases<T, R, true>), dim3(N * (N / 2) / GR), dim3(256), zlds, s,
                           (const void*)delta, w1, yb, m, nn * m, g);
      else
        hipLaunchKernelGGL((k_zpass_ylm_bases<T, R, false>), dim3(N * (N / 2) / GR), dim3(256), zlds, s,
                           (const void*)delta, w1, yb, m, nn * m, g);
      kt_end(CNPC_KT_ZR2C, s);
      CNPC_HIP(hipGetLastError());
      const unsigned blocks = (unsigned)(ft.nf * n * (m / 16));  // a multiple of 8 (n = 256)
      const size_t clds = sizeof(cx<T>) * (N + (size_t)N * 16 + 16 * R) + sizeof(T) * 4 * N;
      kt_begin(CNPC_KT_COL, s);
      hipLaunchKernelGGL((k_colpass_ylm_rr<T, R>), dim3(blocks), dim3(256), clds, s, w1, coef, w2, yb, ft.nf, m);
      kt_end(CNPC_KT_COL, s);
      CNPC_HIP(hipGetLastError());
      ColArgs ax = make_col(n, d->dtype, (int64_t)n * 2 * m * m, (int64_t)4 * m * m * m, (int64_t)2 * m * m,
                            (int64_t)2 * m * m, 2 * m * m, 0, m);
      return colpass<T>(n, -1, w2, out, ax, ft.nf, s);
    }
  }
  if (zspec) {
    set_error("Y_lm transform of z spectra: only the FP32 z-power-bases route takes them");
    return CNPC_EUNSUPPORTED;
  }
  CNPC_TRY(zpass_ylm<T>(n, delta, w1, ft, m, nn * m, g, s));
  return band_forward_yx<T>(n, d->dtype, ft.nf, m, w1, w2, out, s);
}

size_t ylm_r2c_ws_bytes(const cnpc_mesh_desc* d, int nfields, int band) {
  const size_t nn = (size_t)d->n * d->n;
  return (size_t)nfields * (nn * band + (size_t)d->n * 2 * band * band) * 2 * esize(d->dtype);
}

cnpc_status launch_ylm_r2c(const cnpc_mesh_desc* d, int band, int nells, const int32_t* ells,
                           const void* delta, void* out, void* ws, size_t ws_bytes, hipStream_t s,
                           const void* coef, bool delta_zspec) {
  FieldTable ft;
  const int nf = field_table(nells, ells, &ft);
  CNPC_REQUIRE(nf > 0, "too many Y_lm fields (max 32)");
  if (ws_bytes < ylm_r2c_ws_bytes(d, nf, band)) {
    set_error("ylm_r2c workspace too small");
    return CNPC_EWORKSPACE;
  }
  if (d->dtype == CNPC_F64)
    return ylm_r2c_t<double>(d, band, ft, (const double*)delta, (cx<double>*)out, (cx<double>*)ws, nullptr,
                             delta_zspec, s);
  return ylm_r2c_t<float>(d, band, ft, (const float*)delta, (cx<float>*)out, (cx<float>*)ws, (const float*)coef,
                          delta_zspec, s);
}

size_t ylm_coef_bytes(const cnpc_mesh_desc* d, int nells, const int32_t* ells, int band) {
  FieldTable ft;
  if (d->dtype != CNPC_F32 || field_table(nells, ells, &ft) <= 0) return 0;
  const YlmBases yb = ylm_bases(ft, d->los_mode == CNPC_LOS_GLOBAL);
  if (!ylm_bases_route<float>(d->n, band, ft, yb)) return 0;
  return (size_t)ft.nf * d->n * d->n * 4 * sizeof(float);
}

cnpc_status launch_ylm_coef(const cnpc_mesh_desc* d, int nells, const int32_t* ells, int band, void* coef,
                            hipStream_t s) {
  FieldTable ft;
  CNPC_REQUIRE(field_table(nells, ells, &ft) > 0, "too many Y_lm fields (max 32)");
  CNPC_REQUIRE(ylm_coef_bytes(d, nells, ells, band) > 0, "no coefficient table for this transform");
  const Geo g = make_geo(d);
  const YlmBases yb = ylm_bases(ft, g.global_los != 0);
  const int64_t ncoef = (int64_t)ft.nf * d->n * d->n;
  hipLaunchKernelGGL((k_ylm_coef<float>), dim3((unsigned)((ncoef + 255) / 256)), dim3(256), 0, s, ft, yb, d->n, g,
                     (float*)coef);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_ylm_fields(const cnpc_mesh_desc* d, int ell, const void* delta, void* out,
                              hipStream_t s) {
  const int64_t n3 = (int64_t)d->n * d->n * d->n;
  const unsigned nb = (unsigned)std::min<int64_t>((n3 + 255) / 256, 65536);
  if (d->dtype == CNPC_F64)
    hipLaunchKernelGGL((k_ylm_fields<double>), dim3(nb), dim3(256), 0, s, (const double*)delta,
                       (double*)out, d->n, ell, make_geo(d));
  else
    hipLaunchKernelGGL((k_ylm_fields<float>), dim3(nb), dim3(256), 0, s, (const float*)delta,
                       (float*)out, d->n, ell, make_geo(d));
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// ------------------------------------------------------------ interlacing --
// Combine the spectra of meshes A and B: D = 1/2 [SA + exp(-i pi (nx+ny+nz)/N) SB]
// (without interlacing D = SA), modes with a Nyquist component zeroed.  Layout
// of sa/sb: half (m == 0) or band (half-width m).  D * scale_inplace is written
// back into sa; D itself is written to band_out (band half-width mb) when given.
template <typename T>
__global__ void __launch_bounds__(256) k_interlace_combine(cx<T>* sa, const cx<T>* __restrict__ sb,
                                                           int n, int m, cx<T>* band_out, int mb,
                                                           int interlace, T scale_inplace) {
  const int ny_ = m ? 2 * m : n;
  const int nz_ = m ? m : n / 2;
  const int64_t total = (int64_t)ny_ * ny_ * nz_;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % nz_);
    const int jy = (int)((i / nz_) % ny_);
    const int jx = (int)(i / ((int64_t)nz_ * ny_));
    const int nx = m ? band_freq(jx, m) : freq_of(jx, n);
    const int ny = m ? band_freq(jy, m) : freq_of(jy, n);
    cx<T> v = sa[i];
    if (nx == -(n / 2) || ny == -(n / 2)) {
      v = cx<T>{T(0), T(0)};
    } else if (interlace) {
      double sn, cs;
      sincospi(-(double)(nx + ny + kz) / (double)n, &sn, &cs);
      const cx<T> b = sb[i];
      const cx<T> ph = {T(cs), T(sn)};
      v = cscale(cadd(v, cmul(ph, b)), T(0.5));
    }
    sa[i] = cscale(v, scale_inplace);
    if (band_out && nx >= -mb && nx < mb && ny >= -mb && ny < mb && kz < mb) {
      const int bx = nx < 0 ? nx + 2 * mb : nx, by = ny < 0 ? ny + 2 * mb : ny;
      band_out[((int64_t)bx * 2 * mb + by) * mb + kz] = v;
    }
  }
}

size_t deinterlace_ws_bytes(const cnpc_mesh_desc* d) {
  const size_t half = (size_t)d->n * d->n * (d->n / 2) * 2 * esize(d->dtype);
  return 2 * half;
}

size_t deinterlace_band_ws_bytes(const cnpc_mesh_desc* d, int band) {
  const int nb = d->interlace ? 2 : 1;
  const size_t bsz = (size_t)4 * band * band * band;
  return (nb * bsz + fft_ws_elems(d->n, nb, band)) * 2 * esize(d->dtype);
}

// workspace that covers every band (the band-pruned path grows with the band)
size_t deinterlace_ws_max(const cnpc_mesh_desc* d) {
  return std::max(deinterlace_ws_bytes(d), deinterlace_band_ws_bytes(d, d->n / 2));
}

template <typename T>
static cnpc_status deinterlace_t(const cnpc_mesh_desc* d, int band, const T* meshes, cx<T>* spec,
                                 T* delta_int, cx<T>* ws, hipStream_t s) {
  const int n = d->n;
  const int64_t n3 = (int64_t)n * n * n;
  const int il = d->interlace ? 1 : 0;
  const int nb = 1 + il;
  if (delta_int == nullptr || !il) {
    // band-pruned path: only the band of D is needed
    const int64_t bsz = (int64_t)4 * band * band * band;
    cx<T>* sp = ws;                       // [nb][band]
    cx<T>* fws = ws + (int64_t)nb * bsz;  // transform scratch
    CNPC_TRY(fft3d_r2c<T>(n, nb, band, meshes, sp, fws, s));
    const unsigned g = (unsigned)std::min<int64_t>((bsz + 255) / 256, 65536);
    hipLaunchKernelGGL((k_interlace_combine<T>), dim3(g), dim3(256), 0, s, sp, il ? sp + bsz : sp, n,
                       band, spec, band, il, T(1));
    CNPC_HIP(hipGetLastError());
    if (delta_int)
      CNPC_HIP(hipMemcpyAsync(delta_int, meshes, sizeof(T) * n3, hipMemcpyDeviceToDevice, s));
    return CNPC_OK;
  }
  const int64_t hsz = (int64_t)n * n * (n / 2);
  cx<T>* sp = ws;  // [2][half]
  if (has_xpass_interlace(n)) {
    // z and y passes of both phases, then one pass doing their x transforms,
    // the combination, the band copy and the inverse x transform of D / N^3;
    // inverse y and z passes into delta_int (complex view of its N^3 reals)
    CNPC_TRY(ensure_twiddles());
    const int dt = sizeof(T) == 8 ? CNPC_F64 : CNPC_F32;
    const int h = n / 2;
    const int64_t nn = (int64_t)n * n;
    CNPC_TRY(zpass_r2c<T>(n, meshes, sp, 2 * nn, h, s));
    ColArgs ay = make_col(n, dt, (int64_t)n * h, (int64_t)n * h, h, h, h, 0, 0);
    CNPC_TRY(colpass<T>(n, -1, sp, sp, ay, 2 * (int64_t)n, s));
    cx<T>* o = reinterpret_cast<cx<T>*>(delta_int);
    CNPC_TRY(xpass_interlace<T>(n, sp, o, spec, band, T(1.0 / (double)n3), s));
    CNPC_TRY(colpass<T>(n, 1, o, o, ay, (int64_t)n, s));
    return zpass_c2r<T>(n, o, delta_int, nn, h, s);
  }
  CNPC_TRY(fft3d_r2c<T>(n, 2, 0, meshes, sp, nullptr, s));
  const unsigned g = (unsigned)std::min<int64_t>((hsz + 255) / 256, 65536);
  // D / N^3 stays in place for the unnormalised inverse; D itself goes to the band
  hipLaunchKernelGGL((k_interlace_combine<T>), dim3(g), dim3(256), 0, s, sp, sp + hsz, n, 0, spec,
                     band, 1, T(1.0 / (double)n3));
  CNPC_HIP(hipGetLastError());
  return fft3d_c2r<T>(n, 1, 0, sp, delta_int, nullptr, s);
}

// ------------------------------------------- painting + de-interlacing --
// The de-interlacing transforms continued from their z passes (done by the
// fused fold): delta along the full path (y pass, fused x pass with the
// interlace combination and band copy, inverse y and z passes into
// delta_int), N along the band path (y and x band passes, combination).
template <typename T>
static cnpc_status deinterlace_from_z(const cnpc_mesh_desc* d, int band, cx<T>* sp, cx<T>* nw1, cx<T>* nw2,
                                      cx<T>* nsp, cx<T>* spec, T* delta_int, cx<T>* specN, bool zspec_out,
                                      hipStream_t s) {
  const int n = d->n, h = n / 2, m = band;
  const int dt = sizeof(T) == 8 ? CNPC_F64 : CNPC_F32;
  const int64_t nn = (int64_t)n * n, n3 = nn * n;
  ColArgs ay = make_col(n, dt, (int64_t)n * h, (int64_t)n * h, h, h, h, 0, 0);
  CNPC_TRY(colpass<T>(n, -1, sp, sp, ay, 2 * (int64_t)n, s));
  cx<T>* o = reinterpret_cast<cx<T>*>(delta_int);
  CNPC_TRY(xpass_interlace<T>(n, sp, o, spec, band, T(1.0 / (double)n3), s));
  CNPC_TRY(colpass<T>(n, 1, o, o, ay, (int64_t)n, s));
  if (!zspec_out) CNPC_TRY(zpass_c2r<T>(n, o, delta_int, nn, h, s));
  ColArgs by = make_col(n, dt, (int64_t)n * m, (int64_t)2 * m * m, m, m, m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, nw1, nw2, by, 2 * (int64_t)n, s));
  ColArgs bx = make_col(n, dt, (int64_t)n * 2 * m * m, (int64_t)4 * m * m * m, (int64_t)2 * m * m,
                        (int64_t)2 * m * m, 2 * m * m, 0, m);
  CNPC_TRY(colpass<T>(n, -1, nw2, nsp, bx, 2, s));
  const int64_t bsz = (int64_t)4 * m * m * m;
  const unsigned g = (unsigned)std::min<int64_t>((bsz + 255) / 256, 65536);
  hipLaunchKernelGGL((k_interlace_combine<T>), dim3(g), dim3(256), 0, s, nsp, nsp + bsz, n, band, specN, band, 1,
                     T(1));
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// bytes of the scratch that follows the paint workspace
static size_t paint_deinterlace_extra(const cnpc_mesh_desc* d, int band) {
  const size_t n = d->n, m = band, es = esize(d->dtype);
  const size_t sp = 2 * n * n * (n / 2), w1 = 2 * n * n * m, w2 = 2 * n * 2 * m * m, nsp = 2 * 4 * m * m * m;
  return (sp + w1 + w2 + nsp) * 2 * es + 4 * 256;
}

size_t paint_deinterlace_ws_bytes(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, bool weighted, int band) {
  const size_t p = (paint_layout(d, ngal, nran, weighted).total + 255) & ~(size_t)255;
  return p + paint_deinterlace_extra(d, band);
}

cnpc_status launch_paint_deinterlace(const cnpc_mesh_desc* d, int band, const uint32_t* gpos, const float* gw,
                                     int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                                     int sums_lmax, double* gsums, double* rsums, double* norms, void* spec,
                                     void* delta_int, void* specN, void* ws, size_t ws_bytes, hipStream_t s,
                                     bool delta_int_zspec) {
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  if (!has_fold_zr2c(d) || delta_int == nullptr) {
    set_error("painting with fused de-interlacing: unsupported mesh");
    return CNPC_EUNSUPPORTED;
  }
  if (ws_bytes < paint_deinterlace_ws_bytes(d, ngal, nran, weighted, band)) {
    set_error("paint_deinterlace workspace too small");
    return CNPC_EWORKSPACE;
  }
  const size_t ptot = (paint_layout(d, ngal, nran, weighted).total + 255) & ~(size_t)255;
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  const size_t n = d->n, m = band, es = esize(d->dtype);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  unsigned char* sp = w + ptot;
  unsigned char* nw1 = sp + al(2 * n * n * (n / 2) * 2 * es);
  unsigned char* nw2 = nw1 + al(2 * n * n * m * 2 * es);
  unsigned char* nsp = nw2 + al(2 * n * 2 * m * m * 2 * es);
  CNPC_TRY(launch_paint_blocks_zr2c(d, gpos, gw, ngal, rpos, rw, nran, sums_lmax, gsums, rsums, norms, sp, nw1, band,
                                    ws, ptot, s));
  if (d->dtype == CNPC_F64)
    return deinterlace_from_z<double>(d, band, (cx<double>*)sp, (cx<double>*)nw1, (cx<double>*)nw2,
                                      (cx<double>*)nsp, (cx<double>*)spec, (double*)delta_int,
                                      (cx<double>*)specN, delta_int_zspec, s);
  return deinterlace_from_z<float>(d, band, (cx<float>*)sp, (cx<float>*)nw1, (cx<float>*)nw2, (cx<float>*)nsp,
                                   (cx<float>*)spec, (float*)delta_int, (cx<float>*)specN, delta_int_zspec, s);
}

cnpc_status launch_deinterlace(const cnpc_mesh_desc* d, int band, const void* meshes, void* spec,
                               void* delta_int, void* ws, size_t ws_bytes, hipStream_t s) {
  const bool full = delta_int != nullptr && d->interlace;
  if (ws_bytes < (full ? deinterlace_ws_bytes(d) : deinterlace_band_ws_bytes(d, band))) {
    set_error("deinterlace workspace too small");
    return CNPC_EWORKSPACE;
  }
  if (d->dtype == CNPC_F64)
    return deinterlace_t<double>(d, band, (const double*)meshes, (cx<double>*)spec, (double*)delta_int,
                                 (cx<double>*)ws, s);
  return deinterlace_t<float>(d, band, (const float*)meshes, (cx<float>*)spec, (float*)delta_int,
                              (cx<float>*)ws, s);
}

// --------------------------------------------------------- F_l assembly --
template <typename T>
__global__ void __launch_bounds__(256) k_assemble(int n, int m, int ell, int assign,
                                                  const cx<T>* __restrict__ spec0,
                                                  const cx<T>* __restrict__ ylm, cx<T>* __restrict__ F) {
  const int64_t bsz = (int64_t)4 * m * m * m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
    if (n2 == 0 || nx == -(n / 2) || ny == -(n / 2)) {
      F[i] = cx<T>{T(0), T(0)};
      continue;
    }
    const double W = window_1d(nx, n, assign) * window_1d(ny, n, assign) * window_1d(nz, n, assign);
    if (ell == 0) {
      const cx<T> v = spec0[i];
      F[i] = cx<T>{T(v.x / W), T(v.y / W)};
      continue;
    }
    const double inv = 1.0 / sqrt((double)n2);
    T re[5], im[5];
    racah_ylm<T>(ell, T(nx * inv), T(ny * inv), T(nz * inv), re, im);
    cx<T> acc = cscale(ylm[i], re[0]);
    for (int mm = 1; mm <= ell; ++mm) {
      const cx<T> a = ylm[(2 * mm - 1) * bsz + i];
      const cx<T> b = ylm[(2 * mm) * bsz + i];
      acc.x += T(2) * (re[mm] * a.x + im[mm] * b.x);
      acc.y += T(2) * (re[mm] * a.y + im[mm] * b.y);
    }
    F[i] = cx<T>{T(acc.x / W), T(acc.y / W)};
  }
}

cnpc_status launch_assemble(const cnpc_mesh_desc* d, int band, int ell, const void* spec0,
                            const void* ylm, void* F, hipStream_t s) {
  const int64_t bsz = (int64_t)4 * band * band * band;
  const unsigned g = (unsigned)std::min<int64_t>((bsz + 255) / 256, 65536);
  if (d->dtype == CNPC_F64)
    hipLaunchKernelGGL((k_assemble<double>), dim3(g), dim3(256), 0, s, d->n, band, ell, d->assign,
                       (const cx<double>*)spec0, (const cx<double>*)ylm, (cx<double>*)F);
  else
    hipLaunchKernelGGL((k_assemble<float>), dim3(g), dim3(256), 0, s, d->n, band, ell, d->assign,
                       (const cx<float>*)spec0, (const cx<float>*)ylm, (cx<float>*)F);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// ---------------------------------------------------------------- binning --
template <typename T>
__global__ void __launch_bounds__(256) k_bin(BinArgs<T> a, const double* __restrict__ norms,
                                             double* __restrict__ acc_out,
                                             unsigned long long* __restrict__ cnt_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nacc = a.npairs + a.nself + 1;  // + sum |k|
  double* acc = reinterpret_cast<double*>(smem_raw);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(acc + (int64_t)a.nbins * nacc);
  for (int i = threadIdx.x; i < a.nbins * nacc; i += blockDim.x) acc[i] = 0.0;
  for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) cnt[i] = 0ull;
  __syncthreads();
  const int m = a.m, n = a.n;
  const int64_t bsz = (int64_t)4 * m * m * m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    if (nx == -(n / 2) || ny == -(n / 2) || nz == n / 2) continue;
    const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
    if (n2 == 0 || n2 < a.thr[0] || n2 >= a.thr[a.nbins]) continue;
    int lo = 0, hi = a.nbins;  // thr[lo] <= n2 < thr[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (n2 >= a.thr[mid]) lo = mid; else hi = mid;
    }
    const int b = lo;
    const double wgt = nz == 0 ? 1.0 : 2.0;
    double* ab = acc + b * nacc;
    for (int q = 0; q < a.npairs; ++q) {
      const cx<T> fa = a.pa[q][i], fb = a.pb[q][i];
      // Re or Im of F_a F_b^*; for an anti-Hermitian product (odd l) the
      // k and -k halves carry the same imaginary part, so the half-grid
      // weights apply to both
      const double v = ((a.imag >> q) & 1u) ? (double)fa.y * (double)fb.x - (double)fa.x * (double)fb.y
                                            : (double)fa.x * (double)fb.x + (double)fa.y * (double)fb.y;
      atomicAdd(&ab[q], wgt * v);
    }
    if (a.nself) {
      const double kn = sqrt((double)n2);
      const double ux = nx / kn, uy = ny / kn, uz = nz / kn;
      double cxs, ctx, cys, cty, czs, ctz;
      alias_1d(nx, n, a.assign, &cxs, &ctx);
      alias_1d(ny, n, a.assign, &cys, &cty);
      alias_1d(nz, n, a.assign, &czs, &ctz);
      const double C = a.interlace ? 0.5 * (cxs * cys * czs + ctx * cty * ctz) : cxs * cys * czs;
      const double W = window_1d(nx, n, a.assign) * window_1d(ny, n, a.assign) *
                       window_1d(nz, n, a.assign);
      const double cw = C / (W * W);
      for (int q = 0; q < a.nself; ++q) {
        const int l = a.self_ell[q];
        const int base = l == 0 ? 0 : (l == 2 ? 1 : 4);
        double re[5], im[5];
        racah_ylm<double>(l, ux, uy, uz, re, im);
        const double* sb = norms + CNPC_NORM_SBARLM + 2 * base;
        double v = re[0] * sb[0] - im[0] * sb[1];
        for (int mm = 1; mm <= l; ++mm) v += 2.0 * (re[mm] * sb[2 * mm] - im[mm] * sb[2 * mm + 1]);
        atomicAdd(&ab[a.npairs + q], wgt * v * cw);
      }
    }
    atomicAdd(&ab[a.npairs + a.nself], wgt * sqrt((double)n2));
    atomicAdd(&cnt[b], (unsigned long long)(nz == 0 ? 1 : 2));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.nbins * nacc; i += blockDim.x) {
    const double v = acc[i];
    if (v != 0.0) atomicAdd(&acc_out[i], v);
  }
  for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) {
    const unsigned long long c = cnt[i];
    if (c) atomicAdd(&cnt_out[i], c);
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
__global__ void k_zero_i64(int64_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// acc [nbins][nacc] sums -> shell means
__global__ void k_bin_finish(const double* __restrict__ acc, const int64_t* __restrict__ cnt,
                             int nbins, int npairs, int nself, double kf, double* __restrict__ means,
                             double* __restrict__ selfterm, double* __restrict__ keff) {
  const int nacc = npairs + nself + 1;
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const double c = cnt[b] > 0 ? (double)cnt[b] : 1.0;
    for (int q = 0; q < npairs; ++q) means[q * nbins + b] = acc[b * nacc + q] / c;
    for (int q = 0; q < nself; ++q) selfterm[q * nbins + b] = acc[b * nacc + npairs + q] / c;
    if (keff) keff[b] = kf * acc[b * nacc + npairs + nself] / c;
  }
}

size_t bin_ws_doubles(int nbins, int npairs, int nself) {
  return (size_t)nbins * (npairs + nself + 1);
}

template <typename T>
static cnpc_status bin_t(const cnpc_mesh_desc* d, const int64_t* thr, int nbins, int band,
                         int npairs, const void* const* pa, const void* const* pb, uint32_t imag, int nself,
                         const int32_t* self_ells, const double* norms, double* acc, double* means,
                         double* selfterm, int64_t* nmodes, double* keff, hipStream_t s) {
  BinArgs<T> a;
  a.n = d->n;
  a.m = band;
  a.assign = d->assign;
  a.interlace = d->interlace;
  a.nbins = nbins;
  a.npairs = npairs;
  a.nself = nself;
  a.imag = imag;
  for (int b = 0; b <= nbins; ++b) a.thr[b] = thr[b];
  for (int q = 0; q < npairs; ++q) {
    a.pa[q] = (const cx<T>*)pa[q];
    a.pb[q] = (const cx<T>*)pb[q];
  }
  for (int q = 0; q < nself; ++q) a.self_ell[q] = self_ells[q];
  const int nacc = npairs + nself + 1;
  const int64_t nacc_tot = (int64_t)nbins * nacc;
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, acc, nacc_tot);
  CNPC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(256), 0, s, nmodes, (int64_t)nbins);
  CNPC_HIP(hipGetLastError());
  const int64_t bsz = (int64_t)4 * band * band * band;
  const unsigned g = (unsigned)std::min<int64_t>((bsz + 255) / 256, 2048);
  const size_t lds = sizeof(double) * nacc_tot + sizeof(unsigned long long) * nbins;
  kt_begin(CNPC_KT_BIN, s);
  hipLaunchKernelGGL((k_bin<T>), dim3(g), dim3(256), lds, s, a, norms, acc,
                     (unsigned long long*)nmodes);
  kt_end(CNPC_KT_BIN, s);
  CNPC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_bin_finish, dim3(1), dim3(256), 0, s, acc, nmodes, nbins, npairs, nself,
                     2.0 * 3.14159265358979323846 / d->boxsize, means, selfterm, keff);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_bin(const cnpc_mesh_desc* d, const int64_t* thr, int nbins, int band, int npairs,
                       const void* const* pa, const void* const* pb, uint32_t imag, int nself,
                       const int32_t* self_ells, const double* norms, double* acc, double* means,
                       double* selfterm, int64_t* nmodes, double* keff, hipStream_t s) {
  if (d->dtype == CNPC_F64)
    return bin_t<double>(d, thr, nbins, band, npairs, pa, pb, imag, nself, self_ells, norms, acc, means,
                         selfterm, nmodes, keff, s);
  return bin_t<float>(d, thr, nbins, band, npairs, pa, pb, imag, nself, self_ells, norms, acc, means,
                      selfterm, nmodes, keff, s);
}

// ------------------------------------------------------ Yamamoto finalize --
__global__ void k_pk_finalize(int nbins, const double* m00, const double* m02, const double* m04,
                              const double* m22, const double* m42, const double* m44,
                              const double* __restrict__ nm, double* __restrict__ out) {
  const double I22 = nm[CNPC_NORM_I22], N0 = nm[CNPC_NORM_N0];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    const double P0 = m00 ? m00[b] / I22 - N0 : 0.0;
    const double P2 = m02 ? 5.0 * m02[b] / I22 : 0.0;
    const double P4 = m04 ? 9.0 * m04[b] / I22 : 0.0;
    const double P22 = m22 ? 9.0 * m22[b] / I22 - 9.0 / 5.0 * N0 : 0.0;
    const double P42 = m42 ? 13.0 * m42[b] / I22 : 0.0;
    const double P44 = m44 ? 17.0 * m44[b] / I22 - 17.0 / 9.0 * N0 : 0.0;
    out[0 * nbins + b] = P0;
    out[1 * nbins + b] = P2;
    out[2 * nbins + b] = P4;
    out[3 * nbins + b] = P22;
    out[4 * nbins + b] = P42;
    out[5 * nbins + b] = P44;
    out[6 * nbins + b] = 35.0 / 18.0 * P22 - P2 - 3.5 * P0;
    out[7 * nbins + b] = 11.0 / 5.0 * P42 - 52.0 / 63.0 * P4 - 286.0 / 175.0 * P2;
    out[8 * nbins + b] = 1287.0 / 490.0 * P44 - 374.0 / 245.0 * P42 - 3553.0 / 15435.0 * P4 -
                         1326.0 / 8575.0 * P2 - 2431.0 / 490.0 * P0;
  }
}

// one multipole from its shell mean: (2l+1) mean / I22 - delta_l0 N0 (odd l:
// the mean of Im F_0 F_l^*, no shot noise)
__global__ void k_pk_multipole(int nbins, int ell, const double* __restrict__ mean,
                               const double* __restrict__ nm, double* __restrict__ out) {
  const double I22 = nm[CNPC_NORM_I22], N0 = ell == 0 ? nm[CNPC_NORM_N0] : 0.0;
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) out[b] = (2.0 * ell + 1.0) * mean[b] / I22 - N0;
}

cnpc_status launch_pk_multipole(int nbins, int ell, const double* mean, const double* norms, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_pk_multipole, dim3(1), dim3(128), 0, s, nbins, ell, mean, norms, out);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// normalisations of the cross spectrum of tracers A and B: those of A with
// I22 = sqrt(I22_A I22_B) and N0 = 0 (distinct samples share no galaxy)
__global__ void k_cross_norms(const double* __restrict__ na, const double* __restrict__ nb,
                              double* __restrict__ out) {
  for (int i = threadIdx.x; i < CNPC_NORMS_LEN; i += blockDim.x) out[i] = na[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    out[CNPC_NORM_I22] = sqrt(na[CNPC_NORM_I22] * nb[CNPC_NORM_I22]);
    out[CNPC_NORM_N0] = 0.0;
  }
}

cnpc_status launch_cross_norms(const double* na, const double* nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cross_norms, dim3(1), dim3(64), 0, s, na, nb, out);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_pk_finalize(int nbins, const double* m00, const double* m02, const double* m04,
                               const double* m22, const double* m42, const double* m44,
                               const double* norms, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pk_finalize, dim3(1), dim3(256), 0, s, nbins, m00, m02, m04, m22, m42, m44,
                     norms, out);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

}  // namespace cnpc
