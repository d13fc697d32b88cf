// Bispectrum: shell-filtered band c2r, grid contraction C[(a,b),c] = sum_x X_a X_b Y_c,
// normalisation and analytic shot noise (Scoccimarro B_l and TripoSH B_l0l).
#include <cmath>
#include <vector>

#include "bispec.h"

namespace cnpc {

// ------------------------------------------------------------ host maths --
static double legendre_host(int l, double x) {
  if (l == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= l; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Gauss-Legendre nodes / weights on [-1, 1] by Newton iteration on P_n
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// g_l(t) of Lemma 2 from the integral over x in [|t-1|, t+1] of
// x L_l((x^2 + t^2 - 1)/(2 x t)) / (2t), 64-point Gauss-Legendre.
double g_ell_host(int l, double t) {
  if (t == 0.0) return l == 0 ? 1.0 : 0.0;
  static std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(64, gx, gw);
  const double a = fabs(t - 1.0), b = t + 1.0;
  double s = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) {
    const double x = 0.5 * (b - a) * gx[i] + 0.5 * (b + a);
    double c = (x * x + t * t - 1.0) / (2.0 * x * t);
    c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    s += gw[i] * x * legendre_host(l, c);
  }
  return 0.5 * (b - a) * s / (2.0 * t);
}

// exact mode counts per bin over the band (host integer loop)
static std::vector<int64_t> mode_counts(const cnpc_mesh_desc* d, const std::vector<int64_t>& thr,
                                        int nb) {
  std::vector<int64_t> c(nb, 0);
  const int n = d->n, h = n / 2;
  const int64_t tmax = thr[nb];
  int r = 0;
  while ((int64_t)r * r < tmax) ++r;
  for (int nx = -r; nx <= r; ++nx)
    for (int ny = -r; ny <= r; ++ny)
      for (int nz = -r; nz <= r; ++nz) {
        if (nx <= -h || nx >= h || ny <= -h || ny >= h || nz <= -h || nz >= h) continue;
        const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
        if (n2 == 0 || n2 < thr[0] || n2 >= tmax) continue;
        int b = 0;
        while (b + 1 <= nb && n2 >= thr[b + 1]) ++b;
        c[b]++;
      }
  return c;
}

static bool closed(int i, int j, int k) {
  int a = i, b = j, c = k;
  if (a > b) std::swap(a, b);
  if (b > c) std::swap(b, c);
  if (a > b) std::swap(a, b);
  return c <= a + b;
}

static inline int pair_index(int a, int b, int nb) {  // a <= b
  return a * nb - a * (a - 1) / 2 + (b - a);
}

// ---------------------------------------------------------- contraction --
template <typename T>
__global__ void __launch_bounds__(256) k_contract(const T* __restrict__ fields, int64_t npts, int nf,
                                                  int nshell, int npairs, int p0, ContractCols cc,
                                                  const uint32_t* __restrict__ pairs,
                                                  double* __restrict__ partial) {
  constexpr int KT = 128;  // points per LDS tile
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);  // [nf][KT]
  const int p = p0 + threadIdx.x;
  int fa = 0, fb = 0;
  if (p < npairs && pairs) {  // listed pair: a | b << 16
    fa = (int)(pairs[p] & 0xffffu);
    fb = (int)(pairs[p] >> 16);
  } else if (p < npairs) {  // decode pair index -> (a, b), a <= b
    int a = 0, rem = p;
    while (rem >= nshell - a) { rem -= nshell - a; ++a; }
    fa = a;
    fb = a + rem;
  }
  double tot[MAX_COLS];
  T acc[MAX_COLS];
#pragma unroll
  for (int c = 0; c < MAX_COLS; ++c) { tot[c] = 0.0; acc[c] = T(0); }
  const int64_t per_block = (npts + gridDim.x - 1) / gridDim.x;
  const int64_t x0 = (int64_t)blockIdx.x * per_block;
  const int64_t x1 = min(npts, x0 + per_block);
  int tiles_since_flush = 0;
  for (int64_t xb = x0; xb < x1; xb += KT) {
    const int kt = (int)min((int64_t)KT, x1 - xb);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nf * KT; idx += blockDim.x) {
      const int f = idx / KT, k = idx - f * KT;
      tile[idx] = k < kt ? fields[(int64_t)f * npts + xb + k] : T(0);
    }
    __syncthreads();
    if (p < npairs) {
      const T* ta = tile + fa * KT;
      const T* tb = tile + fb * KT;
      for (int k = 0; k < KT; ++k) {
        const T av = ta[k] * tb[k];
#pragma unroll
        for (int c = 0; c < MAX_COLS; ++c)
          if (c < cc.ncols) acc[c] += av * tile[cc.field[c] * KT + k];
      }
    }
    if (++tiles_since_flush == 16) {  // FP32 inside 2048 points, FP64 across
#pragma unroll
      for (int c = 0; c < MAX_COLS; ++c) { tot[c] += (double)acc[c]; acc[c] = T(0); }
      tiles_since_flush = 0;
    }
  }
  if (p < npairs) {
    double* out = partial + ((int64_t)blockIdx.x * npairs + p) * cc.ncols;
#pragma unroll
    for (int c = 0; c < MAX_COLS; ++c)
      if (c < cc.ncols) out[c] = tot[c] + (double)acc[c];
  }
}

// out[i] = sum_b partial[b][i]: a workgroup owns 64 consecutive outputs, its 16
// waves sum interleaved quarters of the rows (four independent chains each),
// then the wave sums are added in a fixed order (deterministic result).
__global__ void __launch_bounds__(1024) k_reduce_blocks(const double* __restrict__ partial, int nblocks,
                                                        int64_t len, double* __restrict__ out) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < len) {
    int b = wv;
    for (; b + 48 < nblocks; b += 64) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += partial[(int64_t)(b + 16 * u) * len + i];
    }
    for (int u = 0; b < nblocks; b += 16, ++u) s[u & 3] += partial[(int64_t)b * len + i];
  }
  red[wv][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wv == 0 && i < len) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k][lane];
    out[i] = t;
  }
}

static cnpc_status reduce_blocks(const double* partial, int nblocks, int64_t len, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_blocks, dim3((unsigned)((len + 63) / 64)), dim3(1024), 0, s, partial, nblocks,
                     len, out);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

constexpr int CONTRACT_BLOCKS = 512;

template <typename T>
cnpc_status contract_valu(const T* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                          double* partial, double* out, hipStream_t s, const uint32_t* pairs, int nlist) {
  const int npairs = pairs ? nlist : nshell * (nshell + 1) / 2;
  const size_t lds = (size_t)nf * 128 * sizeof(T);
  if (lds > lds_limit()) {
    set_error("too many fields for the contraction tile (%d)", nf);
    return CNPC_EUNSUPPORTED;
  }
  for (int p0 = 0; p0 < npairs; p0 += 256) {
    // each launch covers 256 pairs; partials of all launches share the layout
    kt_begin(CNPC_KT_CONTRACT, s);
    hipLaunchKernelGGL((k_contract<T>), dim3(CONTRACT_BLOCKS), dim3(256), lds, s, fields, npts, nf,
                       nshell, npairs, p0, cc, pairs, partial);
    kt_end(CNPC_KT_CONTRACT, s);
    CNPC_HIP(hipGetLastError());
  }
  return reduce_blocks(partial, CONTRACT_BLOCKS, (int64_t)npairs * cc.ncols, out, s);
}

size_t contract_partial_doubles(int nshell, int ncols) {
  // room for the split-BF16 kernel's partials (up to 4 point groups per workgroup)
  return (size_t)CONTRACT_BLOCKS * 4 * nshell * (nshell + 1) / 2 * ncols;
}

// ------------------------------------------------ split-BF16 MFMA contraction --
// C[(a,b), c] = sum_x A[x,(a,b)] B[x,c] with A = X_a X_b formed in FP32 and both
// operands split into bf16 hi + lo; each 32x32 output tile accumulates
// hi*hi + hi*lo + lo*hi with v_mfma_f32_32x32x16_bf16 in FP32 over the
// workgroup's slice of grid points, then the slices are summed in FP64.
// Operand layout of the 32x32x16 bf16 MFMA (64 lanes): lane l holds
// A[l % 32][8 (l / 32) + e] and B[8 (l / 32) + e][l % 32], e = 0..7; the result
// register v of lane l is D[8 (v / 4) + 4 (l / 32) + (v % 4)][l % 32].
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// hi + lo split of 8 floats into packed bf16 by truncation: hi keeps the top 16
// bits of each float (sign, exponent, 7 mantissa bits), lo = v - hi is exact in
// FP32 and is truncated to bf16 in turn, so hi + lo is within 2^-16 |v| of v.
// Two values per v_perm_b32 (the high halves of a pair of words).
__device__ __forceinline__ void split_bf16(const float* v, bf16x8_t& hi, bf16x8_t& lo) {
  u32x4_t h, l;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t b0 = __float_as_uint(v[2 * e]), b1 = __float_as_uint(v[2 * e + 1]);
    const float l0 = v[2 * e] - __uint_as_float(b0 & 0xffff0000u);
    const float l1 = v[2 * e + 1] - __uint_as_float(b1 & 0xffff0000u);
    h[e] = __builtin_amdgcn_perm(b1, b0, 0x07060302u);
    l[e] = __builtin_amdgcn_perm(__float_as_uint(l1), __float_as_uint(l0), 0x07060302u);
  }
  hi = __builtin_bit_cast(bf16x8_t, h);
  lo = __builtin_bit_cast(bf16x8_t, l);
}

constexpr int MF_KC = 256;       // grid points per LDS chunk (= threads per workgroup)
constexpr int MF_PAD = 4;        // row padding (floats) against bank conflicts
constexpr int MF_ROW = MF_KC + MF_PAD;

// ZIN: the fields are given on a 128^3 grid as their z half spectra (rows of
// zm complex values, kz < zm <= 64, layout [field][x][y][kz]); each 256-point
// chunk is the two z rows of one row pair, and its c2r z transform (R1 = 8
// lanes per field, two-for-one) runs in the workgroup before the contraction,
// so the real fields are never stored.
constexpr int MFZ_N = 128, MFZ_R1 = 8, MFZ_R2 = 16, MFZ_MAXF = 24;
// LDS bytes of the c2r staging of ZIN (twiddles + one exchange buffer per field)
constexpr size_t mfz_lds = sizeof(cx<float>) * (MFZ_N + (size_t)MFZ_MAXF * MFZ_R2 * (MFZ_R1 + 1));

// row_fft_q<float, MFZ_R1, MFZ_R2, +1> of the lanes with `active` set; every
// lane of the workgroup passes its two barriers
__device__ __forceinline__ void zrow_c2r(cx<float>* v, int rank, cx<float>* buf, const cx<float>* tw,
                                         bool active) {
  constexpr int R1 = MFZ_R1, R2 = MFZ_R2, Q = R2 / R1;
  if (active) {
    dft_reg<float, R2, 1>(v);
#pragma unroll
    for (int k1 = 0; k1 < R2; ++k1) buf[k1 * (R1 + 1) + rank] = k1 == 0 ? v[k1] : cmul(v[k1], tw[rank * k1]);
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) v[i * R1 + n1] = buf[(rank + R1 * i) * (R1 + 1) + n1];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < Q; ++i) dft_reg<float, R1, 1>(v + i * R1);
  }
}

// The 4 waves of a workgroup form MG = 4 / KG pair groups x KG point groups:
// wave (mg, kg) owns the m-tiles mg*MTW .. mg*MTW+MTW-1 (32 pairs each) and all
// NT n-tiles (32 columns each) for the points kg, kg + KG, ... (16-point steps)
// of every 256-point chunk staged in LDS; the next chunk is prefetched into
// registers meanwhile.  Splitting the points (KG > 1) keeps each operand split
// computed once; splitting the pairs (KG = 1) bounds the accumulators per wave.
template <int MTW, int NT, int KG, int MAXF, bool ZIN = false>
__global__ void __launch_bounds__(256, ZIN ? 3 : 2) k_contract_mfma(const float* __restrict__ fields, int64_t npts,
                                                       int nf, int nshell, int npairs, ContractCols cc,
                                                       const uint32_t* __restrict__ pairs,
                                                       double* __restrict__ partial, int zm = 0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* tile = reinterpret_cast<float*>(smem_raw);  // [nf + 1][MF_ROW]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mg = wave / KG, kg = wave - mg * KG;
  const int zero_row = nf;  // all-zero LDS row for padded pairs / columns
  for (int i = threadIdx.x; i < MF_ROW; i += blockDim.x) tile[zero_row * MF_ROW + i] = 0.f;
  const int grp = lane >> 5, row = lane & 31;
  int offa[MTW], offb[MTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int p = (mg * MTW + i) * 32 + row;
    int a = zero_row, bb = zero_row;
    if (p < npairs && pairs) {
      a = (int)(pairs[p] & 0xffffu);
      bb = (int)(pairs[p] >> 16);
    } else if (p < npairs) {
      int x = 0, rem = p;
      while (rem >= nshell - x) { rem -= nshell - x; ++x; }
      a = x;
      bb = x + rem;
    }
    offa[i] = a * MF_ROW + grp * 8;
    offb[i] = bb * MF_ROW + grp * 8;
  }
  int offc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int j = nt * 32 + row;
    int f = zero_row;
#pragma unroll
    for (int c = 0; c < MAX_COLS; ++c)
      if (c == j && c < cc.ncols) f = cc.field[c];
    offc[nt] = f * MF_ROW + grp * 8;
  }
  f32x16_t acc[MTW][NT];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][nt][v] = 0.f;
  const int64_t per_block = ((npts + gridDim.x - 1) / gridDim.x + MF_KC - 1) / MF_KC * MF_KC;
  const int64_t x0 = (int64_t)blockIdx.x * per_block;
  const int64_t x1 = min(npts, x0 + per_block);
  const float* src = fields + threadIdx.x;
  float pre[MAXF];
  // ZIN: lane group zg (8 lanes) stages field zg; its 16 inputs of the next
  // row pair wait in registers
  constexpr int ZH = MFZ_N / 2;
  const int zg = threadIdx.x / MFZ_R1, zr = threadIdx.x % MFZ_R1;
  cx<float>* ztw = reinterpret_cast<cx<float>*>(smem_raw + sizeof(float) * (nf + 1) * MF_ROW);
  cx<float>* zbuf = ztw + MFZ_N + min(zg, MFZ_MAXF - 1) * (MFZ_R2 * (MFZ_R1 + 1));
  const cx<float>* zsrc =
      reinterpret_cast<const cx<float>*>(fields) + (int64_t)min(zg, nf - 1) * (npts / MFZ_N) * zm;
  cx<float> zv[MFZ_R2];
  // the row pair of chunk xb as one complex sequence A + i B from the half
  // spectra A, B of its rows (clamped straight-line loads; kz >= zm and the
  // Nyquist term are zero)
  auto zload = [&](int64_t xb) {
    const cx<float>* r0 = zsrc + (xb / MFZ_N) * zm;
#pragma unroll
    for (int n2 = 0; n2 < MFZ_R2; ++n2) {
      const int k = zr + MFZ_R1 * n2;
      const int kk = k < ZH ? k : MFZ_N - k;
      const int kc = kk < zm ? kk : zm - 1;
      const cx<float> a = r0[kc], b = r0[zm + kc];
      const cx<float> z = k < ZH ? cx<float>{a.x - b.y, a.y + b.x} : cx<float>{a.x + b.y, b.x - a.y};
      zv[n2] = kk < zm ? z : cx<float>{0.f, 0.f};
    }
  };
  if constexpr (ZIN) {
    load_twiddles<float, MFZ_N, 1>(ztw);
  } else {
    const bool ok = x0 + threadIdx.x < x1;
#pragma unroll
    for (int f = 0; f < MAXF; ++f)
      if (f < nf) pre[f] = ok ? src[(int64_t)f * npts + x0] : 0.f;
  }
  for (int64_t xb = x0; xb < x1; xb += MF_KC) {
    __syncthreads();
    if constexpr (ZIN) {
      zload(xb);  // issued here, not ahead: the registers stay free during the contraction
      zrow_c2r(zv, zr, zbuf, ztw, zg < nf);  // two workgroup barriers
      if (zg < nf) {
        float* t = tile + zg * MF_ROW;
#pragma unroll
        for (int i = 0; i < MFZ_R2 / MFZ_R1; ++i)
#pragma unroll
          for (int k2 = 0; k2 < MFZ_R1; ++k2) {
            const int e = zr + MFZ_R1 * i + MFZ_R2 * k2;
            t[e] = zv[i * MFZ_R1 + k2].x;
            t[MFZ_N + e] = zv[i * MFZ_R1 + k2].y;
          }
      }
    } else {
#pragma unroll
      for (int f = 0; f < MAXF; ++f)
        if (f < nf) tile[f * MF_ROW + threadIdx.x] = pre[f];
    }
    __syncthreads();
    if (xb + MF_KC < x1) {
      const int64_t xn = xb + MF_KC;
      if constexpr (!ZIN) {
        const bool ok = xn + threadIdx.x < x1;
#pragma unroll
        for (int f = 0; f < MAXF; ++f)
          if (f < nf) pre[f] = ok ? src[(int64_t)f * npts + xn] : 0.f;
      }
    }
#pragma unroll
    for (int ks = kg * 16; ks < MF_KC; ks += 16 * KG) {
      bf16x8_t bhi[NT], blo[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        float v[8];
        const float* rc = tile + offc[nt] + ks;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = rc[e];
        split_bf16(v, bhi[nt], blo[nt]);
      }
      // no branches: tiles past the last pair read the zero row, so the
      // accumulators stay in AGPRs across the whole loop
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        float v[8];
        const float* ra = tile + offa[i] + ks;
        const float* rb = tile + offb[i] + ks;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = ra[e] * rb[e];
        bf16x8_t ahi, alo;
        split_bf16(v, ahi, alo);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi[nt], acc[i][nt], 0, 0, 0);
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo[nt], acc[i][nt], 0, 0, 0);
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi[nt], acc[i][nt], 0, 0, 0);
        }
      }
    }
  }
  if constexpr (KG == 4) {
    // the four point groups hold the same tiles: sum them in FP64 through LDS
    // (fixed order) and write one partial per workgroup, coalesced
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem_raw);  // [MTW][NT][16][64]
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      if (kg == k) {
#pragma unroll
        for (int i = 0; i < MTW; ++i)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int idx = ((i * NT + nt) * 16 + v) * 64 + lane;
              red[idx] = (k == 0 ? 0.0 : red[idx]) + (double)acc[i][nt][v];
            }
      }
      __syncthreads();
    }
    double* out = partial + (int64_t)blockIdx.x * npairs * cc.ncols;
    for (int e = threadIdx.x; e < npairs * cc.ncols; e += blockDim.x) {
      const int p = e / cc.ncols, j = e - p * cc.ncols;
      const int r = p & 31;
      const int v = (r >> 3) * 4 + (r & 3), ln = ((r >> 2) & 1) * 32 + (j & 31);
      out[e] = red[(((p >> 5) * NT + (j >> 5)) * 16 + v) * 64 + ln];
    }
    return;
  }
  // one partial per (workgroup, point group)
  double* out = partial + ((int64_t)blockIdx.x * KG + kg) * npairs * cc.ncols;
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int mt = mg * MTW + i;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int j = nt * 32 + row;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int p = mt * 32 + 8 * (v / 4) + 4 * grp + (v % 4);
        if (p < npairs && j < cc.ncols) out[(int64_t)p * cc.ncols + j] = (double)acc[i][nt][v];
      }
    }
  }
}

template <int MTW, int NT, int KG>
static cnpc_status launch_mfma(const float* fields, int64_t npts, int nf, int nshell, int npairs,
                               const ContractCols& cc, const uint32_t* pairs, double* partial, size_t lds,
                               hipStream_t s) {
  if (nf <= 24)
    hipLaunchKernelGGL((k_contract_mfma<MTW, NT, KG, 24>), dim3(CONTRACT_BLOCKS), dim3(256), lds, s,
                       fields, npts, nf, nshell, npairs, cc, pairs, partial);
  else if (nf <= 48)
    hipLaunchKernelGGL((k_contract_mfma<MTW, NT, KG, 48>), dim3(CONTRACT_BLOCKS), dim3(256), lds, s,
                       fields, npts, nf, nshell, npairs, cc, pairs, partial);
  else {
    set_error("split-BF16 contraction supports at most 48 fields");
    return CNPC_EUNSUPPORTED;
  }
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// The split-BF16 contraction of fields given as z half spectra on a 128^3 grid
// (kernel flag ZIN): the default shapes of at most 24 fields, one column tile
// and 4 point groups per workgroup (MTW <= 4).  Returns false (nothing
// launched) where that does not apply.
static bool contract_mfma_z_ok(int nf, int nshell, const ContractCols& cc, int nlist, const uint32_t* pairs) {
  const int npairs = pairs ? nlist : nshell * (nshell + 1) / 2;
  const int mtiles = (npairs + 31) / 32, ntiles = (cc.ncols + 31) / 32;
  const int kg = tune_value(CNPC_TUNE_CONTRACT_KG);
  return nf <= 24 && ntiles == 1 && (kg == 0 || kg == 4) && mtiles <= 4 && fft_register_passes();
}

template <int MTW>
static void launch_mfma_z(const cx<float>* zin, int zm, int64_t npts, int nf, int nshell, int npairs,
                          const ContractCols& cc, const uint32_t* pairs, double* partial, size_t lds,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_contract_mfma<MTW, 1, 4, 24, true>), dim3(CONTRACT_BLOCKS), dim3(256), lds, s,
                     reinterpret_cast<const float*>(zin), npts, nf, nshell, npairs, cc, pairs, partial, zm);
}

static cnpc_status contract_mfma_z(const cx<float>* zin, int zm, int nf, int nshell, const ContractCols& cc,
                                   double* partial, double* out, hipStream_t s, const uint32_t* pairs, int nlist) {
  if (!contract_mfma_z_ok(nf, nshell, cc, nlist, pairs) || zm < 1 || zm > MFZ_N / 2 || nf > MFZ_MAXF) {
    set_error("fused c2r contraction: unsupported shape");
    return CNPC_EUNSUPPORTED;
  }
  const int64_t npts = (int64_t)MFZ_N * MFZ_N * MFZ_N;
  const int npairs = pairs ? nlist : nshell * (nshell + 1) / 2;
  const int mtw = (npairs + 31) / 32;
  const size_t lds_tile = sizeof(float) * (nf + 1) * MF_ROW + mfz_lds;
  const size_t lds_red = (size_t)mtw * 16 * 64 * sizeof(double);
  const size_t lds = lds_tile > lds_red ? lds_tile : lds_red;
  kt_begin(CNPC_KT_CONTRACT, s);
  if (mtw == 1) launch_mfma_z<1>(zin, zm, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  else if (mtw == 2) launch_mfma_z<2>(zin, zm, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  else if (mtw == 3) launch_mfma_z<3>(zin, zm, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  else launch_mfma_z<4>(zin, zm, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  kt_end(CNPC_KT_CONTRACT, s);
  CNPC_HIP(hipGetLastError());
  return reduce_blocks(partial, CONTRACT_BLOCKS, (int64_t)npairs * cc.ncols, out, s);
}

// partial doubles needed by contract_mfma (4 point groups per workgroup at most)
size_t contract_mfma_partial_doubles(int nshell, int ncols) {
  return (size_t)CONTRACT_BLOCKS * 4 * nshell * (nshell + 1) / 2 * ncols;
}

// dispatch of launch_mfma over MTW = 1..MAXMTW for fixed NT, KG
template <int NT, int KG, int MTW>
static cnpc_status launch_mfma_mtw(int mtw, const float* fields, int64_t npts, int nf, int nshell, int npairs,
                                   const ContractCols& cc, const uint32_t* pairs, double* partial, size_t lds,
                                   hipStream_t s) {
  if (mtw == MTW) return launch_mfma<MTW, NT, KG>(fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  if constexpr (MTW > 1)
    return launch_mfma_mtw<NT, KG, MTW - 1>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  set_error("split-BF16 contraction: no kernel for %d tiles per wave", mtw);
  return CNPC_EUNSUPPORTED;
}

cnpc_status contract_mfma(const float* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                          double* partial, double* out, hipStream_t s, const uint32_t* pairs, int nlist) {
  const int npairs = pairs ? nlist : nshell * (nshell + 1) / 2;
  const int mtiles = (npairs + 31) / 32, ntiles = (cc.ncols + 31) / 32;
  if (ntiles > 2 || mtiles > 32) {
    set_error("split-BF16 contraction supports at most 64 columns and 1024 pairs");
    return CNPC_EUNSUPPORTED;
  }
  // staging tile; with 4 point groups also the FP64 reduction of the tiles
  const size_t lds_tile = sizeof(float) * (nf + 1) * MF_ROW;
  // The 4 waves of a workgroup are KG point groups x (4 / KG) pair groups; a
  // wave holds MTW x NT accumulator tiles (<= 8, i.e. <= 128 registers).
  // Default: the most point groups for which the tiles fit (each operand
  // split computed once); tuning knob CNPC_TUNE_CONTRACT_KG overrides.
  auto mtw_for = [&](int kg) { return (mtiles + (4 / kg) - 1) / (4 / kg); };
  int kg = tune_value(CNPC_TUNE_CONTRACT_KG);
  if (kg != 1 && kg != 2 && kg != 4) {
    kg = 4;
    while (kg > 1 && mtw_for(kg) * ntiles > 8) kg >>= 1;
  }
  const int mtw = mtw_for(kg);
  if (mtw * ntiles > 8) {
    set_error("split-BF16 contraction: %d pair tiles x %d column tiles do not fit %d point groups", mtiles,
              ntiles, kg);
    return CNPC_EUNSUPPORTED;
  }
  const size_t lds_red = kg == 4 ? (size_t)mtw * ntiles * 16 * 64 * sizeof(double) : 0;
  const size_t lds = lds_tile > lds_red ? lds_tile : lds_red;
  cnpc_status st;
  kt_begin(CNPC_KT_CONTRACT, s);
  if (ntiles == 1) {
    if (kg == 4) st = launch_mfma_mtw<1, 4, 8>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
    else if (kg == 2) st = launch_mfma_mtw<1, 2, 8>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
    else st = launch_mfma_mtw<1, 1, 8>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  } else {
    if (kg == 4) st = launch_mfma_mtw<2, 4, 4>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
    else if (kg == 2) st = launch_mfma_mtw<2, 2, 4>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
    else st = launch_mfma_mtw<2, 1, 4>(mtw, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  }
  kt_end(CNPC_KT_CONTRACT, s);
  if (st != CNPC_OK) return st;
  return reduce_blocks(partial, kg == 4 ? CONTRACT_BLOCKS : CONTRACT_BLOCKS * kg, (int64_t)npairs * cc.ncols,
                       out, s);
}

// ------------------------------------------ FP32 / FP64 MFMA contraction --
// The same C[r, c] = sum_x X_a X_b Y_c on the matrix cores in the field type:
// FP32 with v_mfma_f32_32x32x2_f32 (32 x 32 output tiles, 2 points per
// instruction), FP64 with v_mfma_f64_16x16x4_f64 (16 x 16 tiles, 4 points).
// Operand layout (TM x TK = 64 lanes): lane l holds A[l % TM][l / TM] and
// B[l / TM][l % TM]; the K index is any bijection onto the points shared by A
// and B, here lane group q = l / TM takes the S consecutive points
// ks + q S .. ks + q S + S - 1 of each step, one per instruction.  Output
// register v of lane l is D[row(v, l)][l % TM]: FP32 32 x 32 row 8 (v / 4) +
// 4 (l / 32) + v % 4, FP64 16 x 16 row 4 v + l / 16.  The pair products X_a X_b are
// formed in the field type; the FP32 accumulators are added into FP64 ones
// every chunk of points, so no FP32 sum runs over more than KC / KG points.
template <typename T>
struct MfmaFp;
template <>
struct MfmaFp<float> {
  static constexpr int TM = 32, TK = 2, NACC = 16;
  typedef float acc_t __attribute__((ext_vector_type(16)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 8 * (v / 4) + 4 * (l / 32) + (v % 4); }
};
template <>
struct MfmaFp<double> {
  static constexpr int TM = 16, TK = 4, NACC = 4;
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 4 * v + l / 16; }
};

// KC: grid points per LDS chunk, 256 or (many FP64 fields: three workgroups per
// CU instead of one) 128; the 256 threads stage 256 / KC fields per point
constexpr int MP_S = 8;     // consecutive points per lane per step

// Wave w of the 4 is point group kg = w % KG of pair group mg = w / KG: it
// owns the MTW m-tiles mg MTW .. and all NT n-tiles, for the steps kg, kg +
// KG, ... of every chunk; one FP64 partial per (workgroup, point group).
template <typename T, int MTW, int NT, int KC>
__global__ void __launch_bounds__(256, 2) k_contract_mfma_fp(const T* __restrict__ fields, int64_t npts, int nf,
                                                          int nshell, int npairs, int kg_n, ContractCols cc,
                                                          const uint32_t* __restrict__ pairs,
                                                          double* __restrict__ partial) {
  using M = MfmaFp<T>;
  constexpr int TM = M::TM, TK = M::TK, NACC = M::NACC, STEP = TK * MP_S;
  constexpr int ROW = KC + (sizeof(T) == 4 ? 4 : 2);  // padded row (elements)
  constexpr int FS = 256 / KC;                            // fields staged per thread and pass
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);  // [nf + 1][ROW]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mg = wave / kg_n, kg = wave - mg * kg_n;
  const int zero_row = nf;
  for (int i = threadIdx.x; i < ROW; i += blockDim.x) tile[zero_row * ROW + i] = T(0);
  const int q = lane / TM, r = lane % TM;
  const int mbase = (int)blockIdx.y * (4 / kg_n) * MTW;  // first m-tile of this workgroup row
  int offa[MTW], offb[MTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int p = (mbase + mg * MTW + i) * TM + r;
    int a = zero_row, bb = zero_row;
    if (p < npairs && pairs) {
      a = (int)(pairs[p] & 0xffffu);
      bb = (int)(pairs[p] >> 16);
    } else if (p < npairs) {
      int x = 0, rem = p;
      while (rem >= nshell - x) { rem -= nshell - x; ++x; }
      a = x;
      bb = x + rem;
    }
    offa[i] = a * ROW + q * MP_S;
    offb[i] = bb * ROW + q * MP_S;
  }
  int offc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int j = nt * TM + r;
    int f = zero_row;
#pragma unroll
    for (int c = 0; c < MAX_COLS; ++c)
      if (c == j && c < cc.ncols) f = cc.field[c];
    offc[nt] = f * ROW + q * MP_S;
  }
  typename M::acc_t acc[MTW][NT];
  double tot[MTW][NT][NACC];
#pragma unroll
  for (int i = 0; i < MTW; ++i)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < NACC; ++v) {
        acc[i][nt][v] = T(0);
        tot[i][nt][v] = 0.0;
      }
  const int64_t per_block = ((npts + gridDim.x - 1) / gridDim.x + KC - 1) / KC * KC;
  const int64_t x0 = (int64_t)blockIdx.x * per_block;
  const int64_t x1 = min(npts, x0 + per_block);
  const int sp = threadIdx.x % KC, sf = threadIdx.x / KC;  // staged point, first field
  for (int64_t xb = x0; xb < x1; xb += KC) {
    __syncthreads();
    {
      const bool ok = xb + sp < x1;
#pragma unroll 8
      for (int f = sf; f < nf; f += FS)
        tile[f * ROW + sp] = ok ? fields[(int64_t)f * npts + xb + sp] : T(0);
    }
    __syncthreads();
    for (int ks = kg * STEP; ks < KC; ks += STEP * kg_n) {
      T bv[NT][MP_S];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < MP_S; ++e) bv[nt][e] = tile[offc[nt] + ks + e];
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        T av[MP_S];
#pragma unroll
        for (int e = 0; e < MP_S; ++e) av[e] = tile[offa[i] + ks + e] * tile[offb[i] + ks + e];
#pragma unroll
        for (int e = 0; e < MP_S; ++e)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[i][nt] = M::mma(av[e], bv[nt][e], acc[i][nt]);
      }
    }
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int i = 0; i < MTW; ++i)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int v = 0; v < NACC; ++v) {
            tot[i][nt][v] += (double)acc[i][nt][v];
            acc[i][nt][v] = T(0);
          }
    }
  }
  double* out = partial + ((int64_t)blockIdx.x * kg_n + kg) * npairs * cc.ncols;
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int mt = mbase + mg * MTW + i;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int j = nt * TM + r;
#pragma unroll
      for (int v = 0; v < NACC; ++v) {
        const int p = mt * TM + M::row(v, lane);
        const double val = sizeof(T) == 4 ? tot[i][nt][v] : (double)acc[i][nt][v];
        if (p < npairs && j < cc.ncols) out[(int64_t)p * cc.ncols + j] = val;
      }
    }
  }
}

// MTW a power of two with MTW x NT <= 4 (FP32) or 16 (FP64) accumulator tiles
// per wave; ny workgroup rows split the m-tiles when one row cannot hold them
template <typename T, int NT, int MTW>
static cnpc_status launch_mfma_fp_mtw(int mtw, int kg, int ny, int kc, const T* fields, int64_t npts, int nf,
                                      int nshell, int npairs, const ContractCols& cc, const uint32_t* pairs,
                                      double* partial, size_t lds, hipStream_t s) {
  if (mtw <= MTW) {
    if (kc == 128)
      hipLaunchKernelGGL((k_contract_mfma_fp<T, MTW, NT, 128>), dim3(CONTRACT_BLOCKS, (unsigned)ny), dim3(256), lds,
                         s, fields, npts, nf, nshell, npairs, kg, cc, pairs, partial);
    else
      hipLaunchKernelGGL((k_contract_mfma_fp<T, MTW, NT, 256>), dim3(CONTRACT_BLOCKS, (unsigned)ny), dim3(256), lds,
                         s, fields, npts, nf, nshell, npairs, kg, cc, pairs, partial);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  }
  if constexpr (sizeof(T) == 8 ? MTW * 2 * NT <= 16 : MTW * 2 * NT <= 4)
    return launch_mfma_fp_mtw<T, NT, MTW * 2>(mtw, kg, ny, kc, fields, npts, nf, nshell, npairs, cc, pairs,
                                              partial, lds, s);
  set_error("MFMA contraction: no kernel for %d tiles per wave", mtw);
  return CNPC_EUNSUPPORTED;
}

template <typename T>
cnpc_status contract_mfma_fp(const T* fields, int64_t npts, int nf, int nshell, const ContractCols& cc,
                             double* partial, double* out, hipStream_t s, const uint32_t* pairs, int nlist) {
  constexpr int TM = MfmaFp<T>::TM;
  constexpr int MAXT = sizeof(T) == 8 ? 16 : 4;  // accumulator tiles per wave
  const int npairs = pairs ? nlist : nshell * (nshell + 1) / 2;
  const int mtiles = (npairs + TM - 1) / TM, ntiles = (cc.ncols + TM - 1) / TM;
  if (ntiles > (sizeof(T) == 8 ? 3 : 2)) {
    set_error("MFMA contraction: too many columns (%d)", cc.ncols);
    return CNPC_EUNSUPPORTED;
  }
  // the most point groups KG whose pair groups fit MAXT tiles per wave (m-tiles
  // per wave rounded up to a power of two); when even KG = 1 does not fit,
  // ny workgroup rows of 4 pair groups x the largest MTW share the m-tiles
  int kg = 4, mtw = 0, ny = 1;
  for (; kg >= 1; kg >>= 1) {
    const int need = (mtiles + (4 / kg) - 1) / (4 / kg);
    mtw = 1;
    while (mtw < need) mtw <<= 1;
    if (mtw * ntiles <= MAXT) break;
  }
  if (kg < 1) {
    kg = 1;
    mtw = 1;
    while (2 * mtw * ntiles <= MAXT) mtw <<= 1;
    ny = (mtiles + 4 * mtw - 1) / (4 * mtw);
  }
  // the 256-point chunk unless its staging tile would keep a CU to one workgroup
  const int kc = sizeof(T) * (size_t)(nf + 1) * (256 + 2) > 56 * 1024 ? 128 : 256;
  const size_t lds = sizeof(T) * (size_t)(nf + 1) * (kc + (sizeof(T) == 4 ? 4 : 2));
  if (lds > lds_limit()) {
    set_error("too many fields for the MFMA contraction tile (%d)", nf);
    return CNPC_EUNSUPPORTED;
  }
  cnpc_status st;
  kt_begin(CNPC_KT_CONTRACT, s);
  if (ntiles == 1) {
    st = launch_mfma_fp_mtw<T, 1, 1>(mtw, kg, ny, kc, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  } else if (ntiles == 2) {
    st = launch_mfma_fp_mtw<T, 2, 1>(mtw, kg, ny, kc, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
  } else {
    if constexpr (sizeof(T) == 8)
      st = launch_mfma_fp_mtw<T, 3, 1>(mtw, kg, ny, kc, fields, npts, nf, nshell, npairs, cc, pairs, partial, lds, s);
    else
      st = CNPC_EUNSUPPORTED;
  }
  kt_end(CNPC_KT_CONTRACT, s);
  if (st != CNPC_OK) return st;
  return reduce_blocks(partial, CONTRACT_BLOCKS * kg, (int64_t)npairs * cc.ncols, out, s);
}

// --------------------------------------------------- shell-filtered c2r --
// X_b = c2r[Phi_b F] for the shells b0..b0+nsh-1 (mask != 0), or G = c2r[F]
// (mask == 0, nsh = 1).  F: band spectrum (half-width m).
template <typename T>
cnpc_status shell_c2r(const cnpc_mesh_desc* d, int m, const cx<T>* F, const int64_t* thr, int nthr,
                      int b0, int nsh, bool mask, T* out, cx<T>* ws, hipStream_t s) {
  const int n = d->n, dt = d->dtype;
  const int64_t nn = (int64_t)n * n;
  cx<T>* w1 = ws;                            // [nsh][n][n][m]
  cx<T>* w2 = ws + (int64_t)nsh * nn * m;    // [nsh][n][2m][m]
  ColArgs ax = make_col(n, dt, 0, (int64_t)n * 2 * m * m, (int64_t)2 * m * m, (int64_t)2 * m * m,
                        2 * m * m, m, 0);
  if (mask) {
    ax.mask_m = m;
    ax.mask_b0 = b0;
    for (int i = 0; i < nthr; ++i) ax.thr[i] = thr[i];
  }
  CNPC_TRY(colpass<T>(n, 1, F, w2, ax, nsh, s));
  ColArgs ay = make_col(n, dt, (int64_t)2 * m * m, (int64_t)n * m, m, m, m, m, 0);
  CNPC_TRY(colpass<T>(n, 1, w2, w1, ay, (int64_t)nsh * n, s));
  CNPC_TRY(zpass_c2r<T>(n, w1, out, (int64_t)nsh * nn, m, s));
  return CNPC_OK;
}

// the x and y passes of shell_c2r alone: X_b's z half spectra into out
// [nsh][n][n][m]; w2: scratch of nsh n 2m m elements
template <typename T>
static cnpc_status shell_xy(const cnpc_mesh_desc* d, int m, const cx<T>* F, const int64_t* thr, int nthr,
                           int b0, int nsh, bool mask, cx<T>* out, cx<T>* w2, hipStream_t s) {
  const int n = d->n, dt = d->dtype;
  ColArgs ax = make_col(n, dt, 0, (int64_t)n * 2 * m * m, (int64_t)2 * m * m, (int64_t)2 * m * m,
                        2 * m * m, m, 0);
  if (mask) {
    ax.mask_m = m;
    ax.mask_b0 = b0;
    for (int i = 0; i < nthr; ++i) ax.thr[i] = thr[i];
  }
  CNPC_TRY(colpass<T>(n, 1, F, w2, ax, nsh, s));
  ColArgs ay = make_col(n, dt, (int64_t)2 * m * m, (int64_t)n * m, m, m, m, m, 0);
  return colpass<T>(n, 1, w2, out, ay, (int64_t)nsh * n, s);
}

size_t shell_c2r_ws_elems(int n, int m, int nsh) {
  const size_t nn = (size_t)n * n;
  return (size_t)nsh * (nn * m + (size_t)n * 2 * m * m);
}

// ------------------------------------------------------------- finalize --
// Cq (TripoSH, optional): exact pair sums of the FFT-method i = j != k term,
// G^3 sum_{q1 in i, q2 in j} Re P(q1 + q2) per shell pair, in place of the
// thin-shell weighted mean of Q_l over k3 bins.
__global__ void k_finalize(FinArgs f, const double* __restrict__ C, const double* __restrict__ Cq,
                           const double* __restrict__ noise,
                           const double* __restrict__ nm, double* __restrict__ raw,
                           double* __restrict__ shot, double* __restrict__ value) {
  const double I33 = nm[CNPC_NORM_I33], Sbar = nm[CNPC_NORM_SBAR];
  const double pre = (2.0 * f.ell + 1.0) / I33;
  const int ne = f.next;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < f.nconf; t += gridDim.x * blockDim.x) {
    const int i = f.cfg[3 * t], j = f.cfg[3 * t + 1], k = f.cfg[3 * t + 2];
    double r, sh = 0.0;
    const int p = f.prow[t];
    if (f.est == CNPC_EST_SCOCCIMARRO) {
      const double c = C[(int64_t)p * f.ncols + i];
      r = pre * c / (f.n3 * (double)f.ntri[t]);
      if (noise) {
        const double* Q = noise;
        const double* H = noise + ne;
        const double* S = noise + 2 * ne;
        double v = (Q[i] - S[i]) + f.aux[2 * t] * (H[j] - S[j]) + f.aux[2 * t + 1] * (H[k] - S[k]);
        if (f.ell == 0) v += Sbar;
        sh = pre * v;
      }
    } else {
      const double c = C[(int64_t)p * f.ncols + 0];
      r = pre * c / (f.n3 * f.counts[i] * f.counts[j]);
      if (noise) {
        const double* Q = noise;
        const double* H = noise + ne;
        const double* S = noise + 2 * ne;
        const double sgn = (f.ell & 1) ? -1.0 : 1.0;
        double v = sgn * (2.0 * f.ell + 1.0) *
                   (f.aux[2 * t] * (H[i] - S[i]) + f.aux[2 * t + 1] * (H[j] - S[j]));
        if (Cq) {
          v += (2.0 * f.ell + 1.0) * Cq[p] / (f.n3 * f.counts[i] * f.counts[j]);
        } else {
          const int c0 = i > j ? i - j : j - i, c1 = i + j;
          double num = 0.0, den = 0.0;
          for (int q = c0; q <= c1; ++q) {
            num += f.wq[q] * (Q[q] - S[q]);
            den += f.wq[q];
          }
          v += (2.0 * f.ell + 1.0) * num / den;
        }
        if (f.ell == 0) v += Sbar;
        sh = v / I33;
      }
    }
    raw[t] = r;
    shot[t] = sh;
    value[t] = r - sh;
  }
}

// ---------------------------------------------------------------- plan --
static cnpc_status device_tables(cnpc_bispec_plan* P) {
  const int nc = P->nconf;
  const size_t npl = P->pairs.size();
  CNPC_HIP(hipMalloc(&P->d_pairs, sizeof(uint32_t) * (npl > 0 ? npl : 1)));
  CNPC_HIP(hipMalloc(&P->d_prow, sizeof(int) * (nc > 0 ? nc : 1)));
  CNPC_HIP(hipMalloc(&P->d_cfg, sizeof(int) * 3 * (nc > 0 ? nc : 1)));
  CNPC_HIP(hipMalloc(&P->d_ntri, sizeof(int64_t) * (nc > 0 ? nc : 1)));
  CNPC_HIP(hipMalloc(&P->d_aux, sizeof(double) * 2 * (nc > 0 ? nc : 1)));
  CNPC_HIP(hipMalloc(&P->d_counts, sizeof(double) * (P->nb > 0 ? P->nb : 1)));
  CNPC_HIP(hipMalloc(&P->d_wq, sizeof(double) * (P->next > 0 ? P->next : 1)));
  return CNPC_OK;
}

static cnpc_status upload_tables(cnpc_bispec_plan* P) {
  const int nc = P->nconf;
  std::vector<double> cnt(P->nb);
  for (int b = 0; b < P->nb; ++b) cnt[b] = (double)P->counts[b];
  CNPC_HIP(hipMemcpy(P->d_pairs, P->pairs.data(), sizeof(uint32_t) * P->pairs.size(), hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_prow, P->prow.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_cfg, P->cfg.data(), sizeof(int) * 3 * nc, hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_ntri, P->ntri.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_aux, P->aux.data(), sizeof(double) * 2 * nc, hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_counts, cnt.data(), sizeof(double) * P->nb, hipMemcpyHostToDevice));
  CNPC_HIP(hipMemcpy(P->d_wq, P->wq.data(), sizeof(double) * P->next, hipMemcpyHostToDevice));
  return CNPC_OK;
}

template <typename T>
__global__ void k_fill_ones(cx<T>* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = cx<T>{T(1), T(0)};
}

// P(q) = F_l(q) N(q)^* - s_l(q) on the band (half-width m) of an n^3 mesh, with
// s_l(q) = Re sum_m y_l^m(qhat) Sbar_l^m C(q) / W(q)^2 the self-pair summand;
// zero at q = 0 and on modes with a Nyquist component.
template <typename T>
__global__ void __launch_bounds__(256) k_noise_product(int n, int m, int assign, int interlace, int ell,
                                                       const cx<T>* __restrict__ Fl,
                                                       const cx<T>* __restrict__ FN0,
                                                       const double* __restrict__ norms,
                                                       cx<T>* __restrict__ P) {
  const int64_t bsz = (int64_t)4 * m * m * m;
  const int base = ell == 0 ? 0 : (ell == 2 ? 1 : 4);
  const double* sb = norms + CNPC_NORM_SBARLM + 2 * base;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
    if (n2 == 0 || nx == -(n / 2) || ny == -(n / 2) || nz == n / 2) {
      P[i] = cx<T>{T(0), T(0)};
      continue;
    }
    const cx<T> a = Fl[i], b = FN0[i];
    double re = (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    const double im = (double)a.y * (double)b.x - (double)a.x * (double)b.y;
    const double kn = sqrt((double)n2);
    double cxs, ctx, cys, cty, czs, ctz;
    alias_1d(nx, n, assign, &cxs, &ctx);
    alias_1d(ny, n, assign, &cys, &cty);
    alias_1d(nz, n, assign, &czs, &ctz);
    const double C = interlace ? 0.5 * (cxs * cys * czs + ctx * cty * ctz) : cxs * cys * czs;
    const double W = window_1d(nx, n, assign) * window_1d(ny, n, assign) * window_1d(nz, n, assign);
    double yr[5], yi[5];
    racah_ylm<double>(ell, nx / kn, ny / kn, nz / kn, yr, yi);
    double sv = yr[0] * sb[0] - yi[0] * sb[1];
    for (int mm = 1; mm <= ell; ++mm) sv += 2.0 * (yr[mm] * sb[2 * mm] - yi[mm] * sb[2 * mm + 1]);
    re -= sv * C / (W * W);
    P[i] = cx<T>{T(re), T(im)};
  }
}

// Band half-width and contraction grid of a bispectrum binning.  Every shell
// field holds modes with |component| <= c_s = floor(sqrt(T_nb - 1)); the
// unfiltered TripoSH field F_l holds the band, |component| <= M - 1.  A sum over
// a G^3 grid of a product of three such fields equals G^3 times the sum over
// exactly closed triangles q1 + q2 + q3 = 0 as soon as no component of
// q1 + q2 + q3 can reach +-G, i.e. G > c1 + c2 + c3; the band layout needs
// G >= 2M.  G is the smallest power of two meeting both, capped at the mesh
// size (where the sum is the mesh's own, as in the plain estimator).
BispecGeom bispec_geometry(const cnpc_mesh_desc* d, const cnpc_kbins* b, int est, int ell) {
  BispecGeom g;
  const double kf = 2.0 * M_PI / d->boxsize;
  const int nb = b->nbins;
  const double kneed = b->kmin + (est == CNPC_EST_TRIPOSH ? (2 * nb - 1) : nb) * b->dk;
  int m = 1;
  while (m < d->n / 2 && (double)m * kf <= kneed) m <<= 1;
  g.band = m;
  std::vector<int64_t> thr(nb + 1);
  bin_thresholds(d, b, thr.data());
  int64_t cs = 0;
  while ((cs + 1) * (cs + 1) <= thr[nb] - 1) ++cs;
  const int64_t c3 = est == CNPC_EST_TRIPOSH ? (int64_t)m - 1 : cs;
  const int64_t need = 2 * cs + c3 + 1;
  int G = 16;
  while (G < d->n && (G < need || G < 2 * m)) G <<= 1;
  g.grid = G;
  if (est == CNPC_EST_TRIPOSH) { g.nfields = nb + 1; g.ncols = 1; }
  else if (ell == 0) { g.nfields = nb; g.ncols = nb; }
  else { g.nfields = 2 * nb; g.ncols = nb; }
  return g;
}

size_t bispec_ws_bytes(const cnpc_mesh_desc* d, const cnpc_kbins* b, int est, int ell) {
  const BispecGeom g = bispec_geometry(d, b, est, ell);
  const int nb = b->nbins, band = g.band;
  const size_t g3 = (size_t)g.grid * g.grid * g.grid;
  const size_t es = esize(d->dtype);
  // run time: fields + c2r scratch for all of them + contraction partials/result
  const size_t run = g.nfields * g3 * es + shell_c2r_ws_elems(g.grid, band, g.nfields) * 2 * es +
                     (contract_partial_doubles(nb, g.ncols) + (size_t)nb * (nb + 1) * g.ncols) * 8;
  // plan time (FP64 indicator fields): ones + fields + scratch + partials
  const size_t bsz = (size_t)4 * band * band * band;
  const size_t plan = bsz * 16 + (size_t)nb * g3 * 8 + shell_c2r_ws_elems(g.grid, band, nb) * 16 +
                      (contract_partial_doubles(nb, nb) + (size_t)nb * (nb + 1) / 2 * nb) * 8;
  return (run > plan ? run : plan) + 4096;
}

static void fields_for(int est, int ell, int nb, ContractCols* cc) {
  if (est == CNPC_EST_TRIPOSH) {
    cc->ncols = 1;
    cc->field[0] = nb;
  } else if (ell == 0) {
    cc->ncols = nb;
    for (int c = 0; c < nb; ++c) cc->field[c] = c;
  } else {
    cc->ncols = nb;
    for (int c = 0; c < nb; ++c) cc->field[c] = nb + c;
  }
}

static unsigned char* align256(unsigned char* p) {
  return reinterpret_cast<unsigned char*>((reinterpret_cast<uintptr_t>(p) + 255) & ~(uintptr_t)255);
}

// Everything of the plan but its allocation; on an error the caller destroys P
// (device tables allocated so far included).
static cnpc_status bispec_plan_build(cnpc_bispec_plan* P, const cnpc_mesh_desc* d, const cnpc_kbins* b, int est,
                                     int ell, int prec, void* ws, size_t ws_bytes, hipStream_t s) {
  P->desc = *d;
  P->bins = *b;
  P->est = est;
  P->ell = ell;
  P->prec = prec;
  P->nb = b->nbins;
  P->thr.resize(P->nb + 1);
  bin_thresholds(d, b, P->thr.data());
  // noise spectra binning: TripoSH needs k3 bins up to |i + j| <= 2 nb - 2
  P->ext = *b;
  if (est == CNPC_EST_TRIPOSH) P->ext.nbins = 2 * P->nb - 1;
  P->next = P->ext.nbins;
  const BispecGeom geo = bispec_geometry(d, b, est, ell);
  const int m = geo.band, G = geo.grid;
  P->band = m;
  P->grid = G;
  P->nfields = geo.nfields;
  P->counts = mode_counts(d, P->thr, P->nb);
  std::vector<int64_t> thr_ext(P->next + 1);
  bin_thresholds(d, &P->ext, thr_ext.data());
  P->counts_ext = mode_counts(d, thr_ext, P->next);
  P->wq.resize(P->next);
  for (int c = 0; c < P->next; ++c) {
    const double kc = b->kmin + (c + 0.5) * b->dk;
    P->wq[c] = (double)P->counts_ext[c] / kc;
  }
  fields_for(est, ell, P->nb, &P->cc);
  // configurations
  const int nb = P->nb;
  std::vector<int> cfg;
  if (est == CNPC_EST_TRIPOSH) {
    for (int i = 0; i < nb; ++i)
      for (int j = i; j < nb; ++j) {
        cfg.push_back(i); cfg.push_back(j); cfg.push_back(-1);
      }
  } else {
    for (int i = 0; i < nb; ++i)
      for (int j = (ell == 0 ? i : 0); j < nb; ++j)
        for (int k = j; k < nb; ++k)
          if (closed(i, j, k)) { cfg.push_back(i); cfg.push_back(j); cfg.push_back(k); }
  }
  const int ncand = (int)cfg.size() / 3;
  std::vector<int64_t> ntri(ncand, 0);
  if (est == CNPC_EST_SCOCCIMARRO) {
    // N_T from FP64 indicator fields, once per binning
    unsigned char* w = align256(reinterpret_cast<unsigned char*>(ws));
    const int64_t g3 = (int64_t)G * G * G;
    const int64_t bsz = (int64_t)4 * m * m * m;
    cx<double>* ones = reinterpret_cast<cx<double>*>(w);
    double* ind = reinterpret_cast<double*>(align256(reinterpret_cast<unsigned char*>(ones + bsz)));
    cx<double>* scr = reinterpret_cast<cx<double>*>(align256(reinterpret_cast<unsigned char*>(ind + (int64_t)nb * g3)));
    double* partial = reinterpret_cast<double*>(align256(reinterpret_cast<unsigned char*>(scr + shell_c2r_ws_elems(G, m, nb))));
    double* Cm = partial + contract_partial_doubles(nb, nb);
    const size_t need = (reinterpret_cast<unsigned char*>(Cm + (size_t)nb * (nb + 1) / 2 * nb) -
                         reinterpret_cast<unsigned char*>(ws));
    if (need > ws_bytes) {
      set_error("bispectrum plan workspace too small: need %zu, got %zu", need, ws_bytes);
      return CNPC_EWORKSPACE;
    }
    cnpc_mesh_desc d64 = *d;
    d64.dtype = CNPC_F64;
    d64.n = G;
    hipLaunchKernelGGL(k_fill_ones<double>, dim3(256), dim3(256), 0, s, ones, bsz);
    CNPC_HIP(hipGetLastError());
    CNPC_TRY(ensure_twiddles());
    CNPC_TRY(shell_c2r<double>(&d64, m, ones, P->thr.data(), nb + 1, 0, nb, true, ind, scr, s));
    ContractCols c2;
    c2.ncols = nb;
    for (int c = 0; c < nb; ++c) c2.field[c] = c;
    CNPC_TRY(contract_valu<double>(ind, g3, nb, nb, c2, partial, Cm, s));
    std::vector<double> hC((size_t)nb * (nb + 1) / 2 * nb);
    CNPC_HIP(hipMemcpyAsync(hC.data(), Cm, sizeof(double) * hC.size(), hipMemcpyDeviceToHost, s));
    CNPC_HIP(hipStreamSynchronize(s));
    for (int t = 0; t < ncand; ++t) {
      const int i = cfg[3 * t], j = cfg[3 * t + 1], k = cfg[3 * t + 2];
      const double v = hC[(size_t)pair_index(j, k, nb) * nb + i] / (double)g3;
      ntri[t] = (int64_t)llround(v);
    }
  }
  // keep configurations with triangles (Scoccimarro) and fill per-config factors
  for (int t = 0; t < ncand; ++t) {
    const int i = cfg[3 * t], j = cfg[3 * t + 1], k = cfg[3 * t + 2];
    if (est == CNPC_EST_SCOCCIMARRO && ntri[t] <= 0) continue;
    P->cfg.push_back(i); P->cfg.push_back(j); P->cfg.push_back(k);
    P->ntri.push_back(est == CNPC_EST_SCOCCIMARRO ? ntri[t] : 0);
    const double ki = b->kmin + (i + 0.5) * b->dk, kj = b->kmin + (j + 0.5) * b->dk;
    if (est == CNPC_EST_SCOCCIMARRO) {
      const double kk = b->kmin + (k + 0.5) * b->dk;
      double mij = (kk * kk - ki * ki - kj * kj) / (2.0 * ki * kj);
      double mik = (kj * kj - ki * ki - kk * kk) / (2.0 * ki * kk);
      mij = mij > 1 ? 1 : (mij < -1 ? -1 : mij);
      mik = mik > 1 ? 1 : (mik < -1 ? -1 : mik);
      P->aux.push_back(legendre_host(ell, mij));
      P->aux.push_back(legendre_host(ell, mik));
    } else {
      const double t_ = ki / kj;
      P->aux.push_back(g_ell_host(ell, t_));
      P->aux.push_back(g_ell_host(ell, 1.0 / t_));
    }
  }
  P->nconf = (int)P->ntri.size();
  // contraction rows: the pairs (j, k) (Scoccimarro, column i) or (i, j)
  // (TripoSH) the kept configurations use, in lexicographic order; for
  // Scoccimarro l = 0 these are the pairs with k <= 2j, about half of all
  {
    std::vector<int> row_of((size_t)nb * (nb + 1) / 2, -1);
    for (int t = 0; t < P->nconf; ++t) {
      const int a = est == CNPC_EST_TRIPOSH ? P->cfg[3 * t] : P->cfg[3 * t + 1];
      const int bb = est == CNPC_EST_TRIPOSH ? P->cfg[3 * t + 1] : P->cfg[3 * t + 2];
      row_of[pair_index(a, bb, nb)] = -2;  // used
    }
    for (int a = 0; a < nb; ++a)
      for (int bb = a; bb < nb; ++bb)
        if (row_of[pair_index(a, bb, nb)] == -2) {
          row_of[pair_index(a, bb, nb)] = (int)P->pairs.size();
          P->pairs.push_back((uint32_t)a | ((uint32_t)bb << 16));
        }
    for (int t = 0; t < P->nconf; ++t) {
      const int a = est == CNPC_EST_TRIPOSH ? P->cfg[3 * t] : P->cfg[3 * t + 1];
      const int bb = est == CNPC_EST_TRIPOSH ? P->cfg[3 * t + 1] : P->cfg[3 * t + 2];
      P->prow.push_back(row_of[pair_index(a, bb, nb)]);
    }
  }
  CNPC_TRY(device_tables(P));
  return upload_tables(P);
}

cnpc_status bispec_plan_create(cnpc_bispec_plan** out, const cnpc_mesh_desc* d, const cnpc_kbins* b,
                               int est, int ell, int prec, void* ws, size_t ws_bytes,
                               hipStream_t s) {
  auto* P = new cnpc_bispec_plan();
  const cnpc_status st = bispec_plan_build(P, d, b, est, ell, prec, ws, ws_bytes, s);
  if (st != CNPC_OK) {
    bispec_plan_destroy(P);
    return st;
  }
  *out = P;
  return CNPC_OK;
}

void bispec_plan_destroy(cnpc_bispec_plan* P) {
  if (!P) return;
  if (P->d_pairs) (void)hipFree(P->d_pairs);
  if (P->d_prow) (void)hipFree(P->d_prow);
  if (P->d_cfg) (void)hipFree(P->d_cfg);
  if (P->d_ntri) (void)hipFree(P->d_ntri);
  if (P->d_aux) (void)hipFree(P->d_aux);
  if (P->d_counts) (void)hipFree(P->d_counts);
  if (P->d_wq) (void)hipFree(P->d_wq);
  if (P->d_wq3) (void)hipFree(P->d_wq3);
  delete P;
}

template <typename T>
static cnpc_status contract_any(const cnpc_bispec_plan* P, const T* fields, int64_t n3, double* partial,
                                double* out, hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (P->prec == CNPC_PREC_BF16X3)
      return contract_mfma(fields, n3, P->nfields, P->nb, P->cc, partial, out, s, P->d_pairs, (int)P->pairs.size());
  }
  return contract_mfma_fp<T>(fields, n3, P->nfields, P->nb, P->cc, partial, out, s, P->d_pairs,
                             (int)P->pairs.size());
}

// FN0 / ind (TripoSH, both or neither): band spectrum of N and the shell
// indicator fields of bispec_indicators; with them the i = j != k shot-noise
// term is the exact pair sum (FFT method) instead of the thin-shell mean.
template <typename T>
static cnpc_status bispec_run_t(const cnpc_bispec_plan* P, const cx<T>* F0, const cx<T>* Fl,
                                const cx<T>* FN0, const T* ind,
                                const double* noise, const double* norms, double* raw, double* shot,
                                double* value, void* ws, size_t ws_bytes, hipStream_t s) {
  // shell fields live on the contraction grid (P->grid)^3, not on the mesh
  cnpc_mesh_desc dg = P->desc;
  dg.n = P->grid;
  const cnpc_mesh_desc* d = &dg;
  const int n = d->n, m = P->band, nb = P->nb;
  const int64_t n3 = (int64_t)n * n * n;
  unsigned char* w = align256(reinterpret_cast<unsigned char*>(ws));
  T* fields = reinterpret_cast<T*>(w);
  cx<T>* scr = reinterpret_cast<cx<T>*>(align256(reinterpret_cast<unsigned char*>(fields + (int64_t)P->nfields * n3)));
  double* partial = reinterpret_cast<double*>(align256(reinterpret_cast<unsigned char*>(scr + shell_c2r_ws_elems(n, m, P->nfields))));
  double* Cm = partial + contract_partial_doubles(nb, P->cc.ncols);
  double* Cq = Cm + (size_t)nb * (nb + 1) / 2 * P->cc.ncols;
  const size_t need = reinterpret_cast<unsigned char*>(Cq + (size_t)nb * (nb + 1) / 2 * P->cc.ncols) -
                      reinterpret_cast<unsigned char*>(ws);
  if (need > ws_bytes) {
    set_error("bispectrum workspace too small: need %zu, got %zu", need, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  CNPC_TRY(ensure_twiddles());
  const int nthr = nb + 1;
  // split BF16 on a 128^3 grid (CNPC_TUNE_SHELL_FUSED 0): the shells' z c2r
  // runs inside the contraction, from their z half spectra in scr
  bool fused = false;
  if constexpr (sizeof(T) == 4)
    fused = P->prec == CNPC_PREC_BF16X3 && n == MFZ_N && m <= MFZ_N / 2 &&
            tune_value(CNPC_TUNE_SHELL_FUSED) != 1 &&
            contract_mfma_z_ok(P->nfields, P->nb, P->cc, (int)P->pairs.size(), P->d_pairs);
  if (fused) {
    if constexpr (sizeof(T) == 4) {
      const int64_t zplane = (int64_t)n * n * m;
      cx<T>* w2 = scr + (int64_t)P->nfields * zplane;
      CNPC_TRY(shell_xy<T>(d, m, F0, P->thr.data(), nthr, 0, nb, true, scr, w2, s));
      if (P->est == CNPC_EST_SCOCCIMARRO && P->ell > 0)
        CNPC_TRY(shell_xy<T>(d, m, Fl, P->thr.data(), nthr, 0, nb, true, scr + (int64_t)nb * zplane, w2, s));
      if (P->est == CNPC_EST_TRIPOSH)
        CNPC_TRY(shell_xy<T>(d, m, Fl, P->thr.data(), nthr, 0, 1, false, scr + (int64_t)nb * zplane, w2, s));
      CNPC_TRY(contract_mfma_z(scr, m, P->nfields, P->nb, P->cc, partial, Cm, s, P->d_pairs,
                               (int)P->pairs.size()));
    }
  } else {
    CNPC_TRY(shell_c2r<T>(d, m, F0, P->thr.data(), nthr, 0, nb, true, fields, scr, s));
    if (P->est == CNPC_EST_SCOCCIMARRO && P->ell > 0)
      CNPC_TRY(shell_c2r<T>(d, m, Fl, P->thr.data(), nthr, 0, nb, true, fields + (int64_t)nb * n3, scr, s));
    if (P->est == CNPC_EST_TRIPOSH)
      CNPC_TRY(shell_c2r<T>(d, m, Fl, P->thr.data(), nthr, 0, 1, false, fields + (int64_t)nb * n3, scr, s));
    CNPC_TRY(contract_any<T>(P, fields, n3, partial, Cm, s));
  }
  const bool exact = ind != nullptr;
  if (exact) {
    // the signal fields are consumed: P(q) goes to the start of the field
    // area (4 m^3 complex values <= one G^3 field, G >= 2m), its c2r to the
    // column slot nb, the cached indicators over slots 0 .. nb-1
    cx<T>* pq = reinterpret_cast<cx<T>*>(fields);
    const int64_t bsz = (int64_t)4 * m * m * m;
    const unsigned gb = (unsigned)std::min<int64_t>((bsz + 255) / 256, 65536);
    hipLaunchKernelGGL((k_noise_product<T>), dim3(gb), dim3(256), 0, s, P->desc.n, m, P->desc.assign,
                       P->desc.interlace, P->ell, Fl, FN0, norms, pq);
    CNPC_HIP(hipGetLastError());
    CNPC_TRY(shell_c2r<T>(d, m, pq, P->thr.data(), nthr, 0, 1, false, fields + (int64_t)nb * n3, scr, s));
    CNPC_HIP(hipMemcpyAsync(fields, ind, sizeof(T) * (size_t)nb * n3, hipMemcpyDeviceToDevice, s));
    CNPC_TRY(contract_any<T>(P, fields, n3, partial, Cq, s));
  }
  FinArgs f;
  f.est = P->est;
  f.ell = P->ell;
  f.nb = nb;
  f.next = P->next;
  f.ncols = P->cc.ncols;
  f.nconf = P->nconf;
  f.n3 = (double)n3;
  f.cfg = P->d_cfg;
  f.prow = P->d_prow;
  f.ntri = P->d_ntri;
  f.aux = P->d_aux;
  f.counts = P->d_counts;
  f.wq = P->d_wq;
  const unsigned g = (unsigned)std::max(1, (P->nconf + 255) / 256);
  hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, f, Cm, exact ? Cq : nullptr, noise, norms, raw,
                     shot, value);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status bispec_run(const cnpc_bispec_plan* P, const void* F0, const void* Fl, const void* FN0,
                       const void* ind, const double* noise, const double* norms, double* raw, double* shot,
                       double* value, void* ws, size_t ws_bytes, hipStream_t s) {
  if (P->desc.dtype == CNPC_F64)
    return bispec_run_t<double>(P, (const cx<double>*)F0, (const cx<double>*)Fl, (const cx<double>*)FN0,
                                (const double*)ind, noise, norms, raw, shot, value, ws, ws_bytes, s);
  return bispec_run_t<float>(P, (const cx<float>*)F0, (const cx<float>*)Fl, (const cx<float>*)FN0,
                             (const float*)ind, noise, norms, raw, shot, value, ws, ws_bytes, s);
}

size_t bispec_indicator_bytes(const cnpc_bispec_plan* P) {
  const size_t g3 = (size_t)P->grid * P->grid * P->grid;
  return (size_t)P->nb * g3 * esize(P->desc.dtype);
}

// I_b = c2r[Phi_b] on the contraction grid, b < nb, in the field type.
template <typename T>
static cnpc_status bispec_indicators_t(const cnpc_bispec_plan* P, T* out, void* ws, size_t ws_bytes,
                                       hipStream_t s) {
  cnpc_mesh_desc dg = P->desc;
  dg.n = P->grid;
  const int m = P->band, nb = P->nb;
  const int64_t bsz = (int64_t)4 * m * m * m;
  unsigned char* w = align256(reinterpret_cast<unsigned char*>(ws));
  cx<T>* ones = reinterpret_cast<cx<T>*>(w);
  cx<T>* scr = reinterpret_cast<cx<T>*>(align256(reinterpret_cast<unsigned char*>(ones + bsz)));
  const size_t need = reinterpret_cast<unsigned char*>(scr + shell_c2r_ws_elems(P->grid, m, nb)) -
                      reinterpret_cast<unsigned char*>(ws);
  if (need > ws_bytes) {
    set_error("indicator workspace too small: need %zu, got %zu", need, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  CNPC_TRY(ensure_twiddles());
  hipLaunchKernelGGL(k_fill_ones<T>, dim3(256), dim3(256), 0, s, ones, bsz);
  CNPC_HIP(hipGetLastError());
  return shell_c2r<T>(&dg, m, ones, P->thr.data(), nb + 1, 0, nb, true, out, scr, s);
}

cnpc_status bispec_indicators(const cnpc_bispec_plan* P, void* out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (P->desc.dtype == CNPC_F64) return bispec_indicators_t<double>(P, (double*)out, ws, ws_bytes, s);
  return bispec_indicators_t<float>(P, (float*)out, ws, ws_bytes, s);
}

}  // namespace cnpc
