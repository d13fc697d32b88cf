// Sugiyama bispectrum multipoles B_l1l2L (tripolar spherical-harmonic
// expansion; section "Sugiyama estimator", eq. sugi_estimator with eq. F_and_G,
// the pairing of eq. sym_sugi, and the shot noise of eqs. S3_sugi_new, q_ells
// and sugi_shot), for l1, l2 <= 4 with l1 + l2 even and L in {0, 2, 4}.
//
// Fields on the contraction grid (all real, c2r of Hermitian band spectra):
//   F_l^m(x; k) = a + i b,  a = c2r[Phi_k F_0 Re y_l^m],  b = c2r[Phi_k F_0 (-Im y_l^m)]
//                 (l even; for l odd a = c2r[-i Phi_k F_0 Im y], b = c2r[-i Phi_k F_0 Re y])
//   G_L^M(x)    = g + i h,  for M >= 0: g = c2r[A_M / W], h = -c2r[B_M / W]
//                 (A_M, B_M: r2c of delta Re / Im y_L^M(xhat)); M < 0 by
//                 G^M = (-1)^M conj(G^-M)
// (the 1/N_k of F is applied at the end).  Each paired sub-configuration adds
//   Re[F1 F2 G] = a1 (a2 g - b2 h) + b1 (-b2 g - a2 h)
// as up to two GEMMs over grid points, sum_x P_i W_j with P = a1 or b1 (the
// k1 shells) and W the pointwise products of the k2 shells with g and h.
#include "bispec.h"

namespace cnpc {

// ------------------------------------------------------------- host math --
static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Wigner 3j symbol, Racah formula
static double wigner3j_host(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0 || j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
  const double tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
  const double pref = tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) * fact(j3 + m3) *
                      fact(j3 - m3);
  double s = 0.0;
  for (int k = 0; k <= j1 + j2 + j3; ++k) {
    const int d[6] = {k, j1 + j2 - j3 - k, j1 - m1 - k, j2 + m2 - k, j3 - j2 + m1 + k, j3 - j1 - m2 + k};
    bool ok = true;
    double den = 1.0;
    for (int t = 0; t < 6; ++t) {
      if (d[t] < 0) { ok = false; break; }
      den *= fact(d[t]);
    }
    if (ok) s += ((k & 1) ? -1.0 : 1.0) / den;
  }
  return (((j1 - j2 - m3) % 2 + 2) % 2 ? -1.0 : 1.0) * std::sqrt(pref) * s;
}

// Racah-normalised associated Legendre function y_l^n(theta, phi = 0) with
// cos theta = mu: sqrt((l-n)!/(l+n)!) P_l^n(mu), Condon-Shortley phase in
// P_l^n, and y_l^-n = (-1)^n y_l^n on phi = 0.
static double racah_plm_host(int l, int n, double mu) {
  const int an = std::abs(n);
  if (an > l) return 0.0;
  const double st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
  double pmm = 1.0;  // P_m^m = (-1)^m (2m-1)!! st^m
  for (int i = 1; i <= an; ++i) pmm *= -(2.0 * i - 1.0) * st;
  double p = pmm;
  if (l > an) {
    double pm1 = mu * (2.0 * an + 1.0) * pmm;  // P_{m+1}^m
    p = pm1;
    for (int ll = an + 2; ll <= l; ++ll) {
      const double pn = ((2.0 * ll - 1.0) * mu * pm1 - (ll + an - 1.0) * pmm) / (ll - an);
      pmm = pm1;
      pm1 = pn;
      p = pn;
    }
  }
  const double y = std::sqrt(fact(l - an) / fact(l + an)) * p;
  return (n < 0 && (an & 1)) ? -y : y;
}

// q_l1l2L(k1, k2, k3) with the cosines of the closed triangle
static double q_factor_host(int l1, int l2, int L, double k1, double k2, double k3) {
  auto clip = [](double x) { return x > 1.0 ? 1.0 : (x < -1.0 ? -1.0 : x); };
  const double mu13 = clip((k2 * k2 - k1 * k1 - k3 * k3) / (2.0 * k1 * k3));
  const double mu23 = clip((k1 * k1 - k2 * k2 - k3 * k3) / (2.0 * k2 * k3));
  double s = 0.0;
  const int nm = std::min(l1, l2);
  for (int n = -nm; n <= nm; ++n) {
    const double w = wigner3j_host(l1, l2, L, n, -n, 0);
    if (w == 0.0) continue;
    s += ((n & 1) ? -1.0 : 1.0) * racah_plm_host(l1, n, mu13) * racah_plm_host(l2, -n, mu23) * w;
  }
  return s;
}

// --------------------------------------------------------------- kernels --
// Band spectrum of the real (part 0) or imaginary (part 1) part of
// F_l^m(x) = sum_q e^{iq.x} y_l^m*(qhat) F0(q) (F0 Hermitian):
//   l even: F0 Re y (part 0), -F0 Im y (part 1)
//   l odd:  -i F0 Im y (part 0), -i F0 Re y (part 1)
// each Hermitian, so that a c2r gives the real field.
template <typename T>
__global__ void __launch_bounds__(256) k_weight_ylm(int m, int ell, int em, int part,
                                                    const cx<T>* __restrict__ F0, cx<T>* __restrict__ out) {
  const int64_t bsz = (int64_t)4 * m * m * m;
  const int am = em < 0 ? -em : em;
  const double sg = (em < 0 && (am & 1)) ? -1.0 : 1.0;  // y^-m = (-1)^m conj(y^m)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    const int64_t n2 = (int64_t)nx * nx + (int64_t)ny * ny + (int64_t)nz * nz;
    double wgt = 0.0;
    if (n2 > 0) {
      const double kn = sqrt((double)n2);
      double yr[5], yi[5];
      racah_ylm<double>(ell, nx / kn, ny / kn, nz / kn, yr, yi);
      const double re = sg * yr[am], im = (em < 0 ? -sg : sg) * yi[am];
      wgt = (ell & 1) ? (part == 0 ? im : re) : (part == 0 ? re : -im);
    }
    const cx<T> f = F0[i];
    if (ell & 1)  // times -i
      out[i] = cx<T>{T(wgt * (double)f.y), T(-wgt * (double)f.x)};
    else
      out[i] = cx<T>{T(wgt * (double)f.x), T(wgt * (double)f.y)};
  }
}

// out = scale * in / W(q) on the band of an n^3 mesh; zero at q = 0 and on
// modes with a Nyquist component
template <typename T>
__global__ void __launch_bounds__(256) k_div_window(int n, int m, int assign, double scale,
                                                    const cx<T>* __restrict__ in, cx<T>* __restrict__ out) {
  const int64_t bsz = (int64_t)4 * m * m * m;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    const bool zero = (nx == 0 && ny == 0 && nz == 0) || nx == -(n / 2) || ny == -(n / 2) || nz == n / 2;
    if (zero) {
      out[i] = cx<T>{T(0), T(0)};
      continue;
    }
    const double W = window_1d(nx, n, assign) * window_1d(ny, n, assign) * window_1d(nz, n, assign);
    const cx<T> a = in[i];
    out[i] = cx<T>{T(scale * (double)a.x / W), T(scale * (double)a.y / W)};
  }
}

// Line-of-sight noise product of the FFT-method i = j != k term:
// out = scale * [(src / W if div else src) * conj(FN0) - sgn * norms[sidx] * C / W^2]
// on the band; zero at q = 0 and on modes with a Nyquist component
template <typename T>
__global__ void __launch_bounds__(256) k_los_noise(int n, int m, int assign, int interlace, int div,
                                                   const cx<T>* __restrict__ src, const cx<T>* __restrict__ FN0,
                                                   const double* __restrict__ norms, int sidx, double sgn,
                                                   double scale, cx<T>* __restrict__ out) {
  const int64_t bsz = (int64_t)4 * m * m * m;
  const double sb = sgn * norms[sidx];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < bsz;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(i % m);
    const int jy = (int)((i / m) % (2 * m));
    const int jx = (int)(i / ((int64_t)2 * m * m));
    const int nx = band_freq(jx, m), ny = band_freq(jy, m), nz = kz;
    const bool zero = (nx == 0 && ny == 0 && nz == 0) || nx == -(n / 2) || ny == -(n / 2) || nz == n / 2;
    if (zero) {
      out[i] = cx<T>{T(0), T(0)};
      continue;
    }
    const double W = window_1d(nx, n, assign) * window_1d(ny, n, assign) * window_1d(nz, n, assign);
    double cxs, ctx, cys, cty, czs, ctz;
    alias_1d(nx, n, assign, &cxs, &ctx);
    alias_1d(ny, n, assign, &cys, &cty);
    alias_1d(nz, n, assign, &czs, &ctz);
    const double C = interlace ? 0.5 * (cxs * cys * czs + ctx * cty * ctz) : cxs * cys * czs;
    const cx<T> a = src[i], b = FN0[i];
    const double ar = div ? (double)a.x / W : (double)a.x, ai = div ? (double)a.y / W : (double)a.y;
    const double re = ar * (double)b.x + ai * (double)b.y - sb * C / (W * W);
    const double im = ai * (double)b.x - ar * (double)b.y;
    out[i] = cx<T>{T(scale * re), T(scale * im)};
  }
}

template <typename T>
__global__ void k_fill_real(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// W_j = c1 X_j Z1 + c2 Y_j Z2 for the nb shells j (a term is left out when
// its field pointer is null)
template <typename T>
__global__ void __launch_bounds__(256) k_sugi_w(int64_t n3, int nb, const T* __restrict__ X,
                                                const T* __restrict__ Z1, double c1, const T* __restrict__ Y,
                                                const T* __restrict__ Z2, double c2, T* __restrict__ W) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n3; x += (int64_t)gridDim.x * blockDim.x) {
    const T z1 = X ? Z1[x] : T(0), z2 = Y ? Z2[x] : T(0);
    for (int j = 0; j < nb; ++j) {
      T v = T(0);
      if (X) v += T(c1) * X[(int64_t)j * n3 + x] * z1;
      if (Y) v += T(c2) * Y[(int64_t)j * n3 + x] * z2;
      W[(int64_t)j * n3 + x] = v;
    }
  }
}

__device__ __forceinline__ int pair_of(int a, int b, int ns) {  // a <= b
  return a * ns - a * (a - 1) / 2 + (b - a);
}

// acc[i][j] += coef * v_ij with (mode 0) v_ij = C_ij, row i (the pair of
// field i of P with the all-ones field nb) against column j; (mode 1) C_ij +
// C_ji; (mode 2) the pair (min(i, j), max(i, j)) of the nb shell fields of P
// (all pairs, lexicographic rows) against their one column
__global__ void k_sugi_accum(const double* __restrict__ C, int nb, int mode, double coef,
                             double* __restrict__ acc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nb) return;
  const int i = t / nb, j = t - i * nb;
  double v;
  if (mode == 2) {
    v = C[pair_of(i < j ? i : j, i < j ? j : i, nb)];
  } else {  // rows of the pairs (i, nb): row i
    v = C[(int64_t)i * nb + j];
    if (mode == 1) v += C[(int64_t)j * nb + i];
  }
  acc[t] += coef * v;
}

struct SugiFin {
  int l1, l2, L, nb, next;
  double hn, n3;
  const double* counts;
  const double* wq3;
};

// acc2 (optional): the FFT-method i = j != k sums, in place of the q-weighted
// thin-shell term
__global__ void k_sugi_finalize(SugiFin f, const double* __restrict__ acc, const double* __restrict__ acc2,
                                const double* __restrict__ noise,
                                const double* __restrict__ nm, double* __restrict__ raw,
                                double* __restrict__ shot, double* __restrict__ value) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f.nb * f.nb) return;
  const int i = t / f.nb, j = t - i * f.nb;
  const double I33 = nm[CNPC_NORM_I33], Sbar = nm[CNPC_NORM_SBAR];
  const double r = f.hn / I33 * acc[t] / (f.n3 * f.counts[i] * f.counts[j]);
  double sh = 0.0;
  if (noise) {
    const int ne = f.next;
    const double* Q = noise;
    const double* H = noise + ne;
    const double* S = noise + 2 * ne;
    double v = 0.0;
    if (f.l1 == 0 && f.l2 == 0 && f.L == 0) v += Sbar;
    if (f.l1 == f.L && f.l2 == 0) v += (2.0 * f.L + 1.0) * (H[i] - S[i]);
    if (f.l2 == f.L && f.l1 == 0) v += (2.0 * f.L + 1.0) * (H[j] - S[j]);
    if (acc2) {
      v += f.hn * acc2[t] / (f.n3 * f.counts[i] * f.counts[j]);
    } else {
      const double* w = f.wq3 + (int64_t)t * ne;
      double q = 0.0;
      for (int c = 0; c < ne; ++c) q += w[c] * (Q[c] - S[c]);
      v += f.hn * q;
    }
    sh = v / I33;
  }
  raw[t] = r;
  shot[t] = sh;
  value[t] = r - sh;
}

// ------------------------------------------------------------------ plan --
static size_t sugi_ws_bytes(const cnpc_mesh_desc* d, const cnpc_kbins* b) {
  const BispecGeom g = bispec_geometry(d, b, CNPC_EST_TRIPOSH, 0);
  const int nb = b->nbins, m = g.band;
  const size_t g3 = (size_t)g.grid * g.grid * g.grid, es = esize(d->dtype);
  const size_t np1 = (size_t)(nb + 1) * (nb + 2) / 2;
  return (size_t)(4 * nb + 3) * g3 * es + (size_t)2 * 4 * m * m * m * 2 * es +
         shell_c2r_ws_elems(g.grid, m, nb) * 2 * es +
         (contract_partial_doubles(nb + 1, nb) + np1 * nb + (size_t)2 * nb * nb) * 8 + 8192;
}

static cnpc_status sugi_plan_create(cnpc_bispec_plan** out, const cnpc_mesh_desc* d, const cnpc_kbins* b, int l1,
                                    int l2, int L, int prec) {
  auto* P = new cnpc_bispec_plan();
  P->desc = *d;
  P->bins = *b;
  P->est = CNPC_EST_SUGIYAMA;
  P->ell = L;
  P->prec = prec;
  P->l1 = l1;
  P->l2 = l2;
  P->L = L;
  P->nb = b->nbins;
  P->thr.resize(P->nb + 1);
  bin_thresholds(d, b, P->thr.data());
  P->ext = *b;
  P->ext.nbins = 2 * P->nb - 1;
  P->next = P->ext.nbins;
  const BispecGeom geo = bispec_geometry(d, b, CNPC_EST_TRIPOSH, 0);
  P->band = geo.band;
  P->grid = geo.grid;
  P->nfields = 2 * P->nb + 2;
  P->counts = mode_counts(d, P->thr, P->nb);
  std::vector<int64_t> thr_ext(P->next + 1);
  bin_thresholds(d, &P->ext, thr_ext.data());
  P->counts_ext = mode_counts(d, thr_ext, P->next);
  P->wq.resize(P->next);
  for (int c = 0; c < P->next; ++c) P->wq[c] = (double)P->counts_ext[c] / (b->kmin + (c + 0.5) * b->dk);
  // paired sub-configurations: M < 0, or M = 0 with m1 <= 0; eta = 2 except
  // (0, 0, 0).  For l1 = l2 (section "Sugiyama estimator", symmetries between
  // and within sub-configurations): (m2, m1, M) gives the transpose in (k1, k2)
  // of (m1, m2, M) with the same 3j symbol (L even), so only m1 < m2 is kept
  // and added with its transpose (flag 1); (m, -m, 0) is symmetric in (k1, k2)
  // and needs the fields of one leg only (flag 2).
  for (int M = -L; M <= 0; ++M)
    for (int m1 = -l1; m1 <= l1; ++m1) {
      const int m2 = -m1 - M;
      if (std::abs(m2) > l2 || (M == 0 && m1 > 0)) continue;
      const double w = wigner3j_host(l1, l2, L, m1, m2, M);
      if (w == 0.0) continue;
      int flag = 0;
      if (l1 == l2) {
        if (M == 0) flag = 2;
        else if (m1 > m2) continue;
        else if (m1 < m2) flag = 1;
      }
      P->sub.push_back(m1);
      P->sub.push_back(m2);
      P->sub.push_back(M);
      P->sub.push_back(flag);
      P->subw.push_back((m1 == 0 && m2 == 0 && M == 0) ? w : 2.0 * w);
    }
  P->hn = wigner3j_host(l1, l2, L, 0, 0, 0) * (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1);
  // every (k1, k2) pair of shells
  const int nb = P->nb;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      P->cfg.push_back(i); P->cfg.push_back(j); P->cfg.push_back(-1);
      P->ntri.push_back(0);
      P->aux.push_back(0.0); P->aux.push_back(0.0);
    }
  P->nconf = nb * nb;
  // k3 weights of the i = j != k term: q(k1, k2, k_c) N_c/k_c / sum_c N_c/k_c
  std::vector<double> wq3((size_t)nb * nb * P->next, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      const int c0 = std::abs(i - j), c1 = i + j;
      double den = 0.0;
      for (int c = c0; c <= c1; ++c) den += P->wq[c];
      const double ki = b->kmin + (i + 0.5) * b->dk, kj = b->kmin + (j + 0.5) * b->dk;
      for (int c = c0; c <= c1; ++c) {
        const double kc = b->kmin + (c + 0.5) * b->dk;
        wq3[((size_t)i * nb + j) * P->next + c] = q_factor_host(l1, l2, L, ki, kj, kc) * P->wq[c] / den;
      }
    }
  // rows of the cross-leg contraction: the pairs (i, nb), shell field i times
  // the all-ones field
  for (int i = 0; i < nb; ++i) P->pairs.push_back((uint32_t)i | ((uint32_t)nb << 16));
  P->prow.assign(P->nconf, 0);
  cnpc_status st = device_tables(P);
  if (st == CNPC_OK) st = upload_tables(P);
  if (st == CNPC_OK) {
    if (hipMalloc(&P->d_wq3, sizeof(double) * wq3.size()) != hipSuccess ||
        hipMemcpy(P->d_wq3, wq3.data(), sizeof(double) * wq3.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("device tables of the Sugiyama plan failed");
      st = CNPC_EHIP;
    }
  }
  if (st != CNPC_OK) {
    bispec_plan_destroy(P);
    return st;
  }
  *out = P;
  return CNPC_OK;
}

// ------------------------------------------------------------------- run --
// FN0 (optional): band spectrum of N_0 / W; with it the i = j != k noise
// term is the FFT method's (a second pass over the sub-configurations with
// harmonic shell indicators and the line-of-sight noise product)
template <typename T>
static cnpc_status sugi_run_t(const cnpc_bispec_plan* P, const cx<T>* F0, const cx<T>* ylm, const cx<T>* FN0,
                              const double* noise, const double* norms, double* raw, double* shot, double* value,
                              void* ws, size_t ws_bytes, hipStream_t s) {
  cnpc_mesh_desc dg = P->desc;
  dg.n = P->grid;
  const int G = P->grid, m = P->band, nb = P->nb;
  const int64_t n3 = (int64_t)G * G * G, bsz = (int64_t)4 * m * m * m;
  const int np1 = (nb + 1) * (nb + 2) / 2;
  unsigned char* w = align256(reinterpret_cast<unsigned char*>(ws));
  // [P: nb][ones][W: nb] (the contraction's fields), then [Qa: nb][Qb: nb][g][h]
  T* fields = reinterpret_cast<T*>(w);
  cx<T>* spec = reinterpret_cast<cx<T>*>(align256(reinterpret_cast<unsigned char*>(fields + (int64_t)(4 * nb + 3) * n3)));
  cx<T>* ones = reinterpret_cast<cx<T>*>(align256(reinterpret_cast<unsigned char*>(spec + bsz)));
  cx<T>* scr = reinterpret_cast<cx<T>*>(align256(reinterpret_cast<unsigned char*>(ones + bsz)));
  double* partial = reinterpret_cast<double*>(align256(reinterpret_cast<unsigned char*>(scr + shell_c2r_ws_elems(G, m, nb))));
  double* Cm = partial + contract_partial_doubles(nb + 1, nb);
  double* acc = Cm + (size_t)np1 * nb;
  double* acc2 = acc + (size_t)nb * nb;
  const size_t need = reinterpret_cast<unsigned char*>(acc2 + (size_t)nb * nb) - reinterpret_cast<unsigned char*>(ws);
  if (need > ws_bytes) {
    set_error("Sugiyama workspace too small: need %zu, got %zu", need, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  CNPC_TRY(ensure_twiddles());
  const unsigned gb = (unsigned)std::min<int64_t>((bsz + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, s, acc, (int64_t)2 * nb * nb);
  CNPC_HIP(hipGetLastError());
  T* slotP = fields;
  T* slotOne = fields + (int64_t)nb * n3;
  T* slotW = slotOne + n3;
  T* slotQa = slotW + (int64_t)nb * n3;
  T* slotQb = slotQa + (int64_t)nb * n3;
  T* slotG = slotQb + (int64_t)nb * n3;
  T* slotH = slotG + n3;
  hipLaunchKernelGGL((k_fill_real<T>), dim3(1024), dim3(256), 0, s, slotOne, n3, T(1));
  CNPC_HIP(hipGetLastError());
  const unsigned gw = (unsigned)std::min<int64_t>((n3 + 255) / 256, 8192);
  // leg field (l, m, part) of every shell into a slot, from F_0 (signal) or
  // from ones (harmonic shell indicators of the FFT-method noise)
  const cx<T>* legsrc = F0;
  auto load_leg = [&](T* slot, int ell, int em, int part) -> cnpc_status {
    hipLaunchKernelGGL((k_weight_ylm<T>), dim3(gb), dim3(256), 0, s, m, ell, em, part, legsrc, spec);
    CNPC_HIP(hipGetLastError());
    return shell_c2r<T>(&dg, m, spec, P->thr.data(), nb + 1, 0, nb, true, slot, scr, s);
  };
  // one unmasked band c2r of scale * in / W into a slot
  auto load_los = [&](T* slot, const cx<T>* in, double scale) -> cnpc_status {
    hipLaunchKernelGGL((k_div_window<T>), dim3(gb), dim3(256), 0, s, P->desc.n, m, P->desc.assign, scale, in, spec);
    CNPC_HIP(hipGetLastError());
    return shell_c2r<T>(&dg, m, spec, P->thr.data(), nb + 1, 0, 1, false, slot, scr, s);
  };
  // sum_x P_i W_j as a GEMM over grid points: the nb + 1 "shell" fields are
  // P and the all-ones field, the nb columns W (W_j = c1 X_j Z1 + c2 Y_j Z2)
  double* accum = acc;
  auto contract_add = [&](const T* X, const T* Z1, double c1, const T* Y, const T* Z2, double c2, double coef,
                          int transpose) -> cnpc_status {
    hipLaunchKernelGGL((k_sugi_w<T>), dim3(gw), dim3(256), 0, s, n3, nb, X, Z1, c1, Y, Z2, c2, slotW);
    CNPC_HIP(hipGetLastError());
    ContractCols cc;
    cc.ncols = nb;
    for (int j = 0; j < nb; ++j) cc.field[j] = nb + 1 + j;
    if constexpr (sizeof(T) == 4) {
      if (P->prec == CNPC_PREC_BF16X3) {
        CNPC_TRY(contract_mfma(fields, n3, 2 * nb + 1, nb + 1, cc, partial, Cm, s, P->d_pairs, nb));
      } else {
        CNPC_TRY(contract_mfma_fp<T>(fields, n3, 2 * nb + 1, nb + 1, cc, partial, Cm, s, P->d_pairs, nb));
      }
    } else {
      CNPC_TRY(contract_mfma_fp<T>(fields, n3, 2 * nb + 1, nb + 1, cc, partial, Cm, s, P->d_pairs, nb));
    }
    hipLaunchKernelGGL(k_sugi_accum, dim3((nb * nb + 255) / 256), dim3(256), 0, s, Cm, nb, transpose, coef, accum);
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  };
  // sum_x P_i P_j g over the pairs i <= j of the nb fields of P, with g copied
  // into the all-ones slot for the call (one column; restored afterwards)
  auto contract_self = [&](double coef) -> cnpc_status {
    CNPC_HIP(hipMemcpyAsync(slotOne, slotG, sizeof(T) * (size_t)n3, hipMemcpyDeviceToDevice, s));
    ContractCols cc;
    cc.ncols = 1;
    cc.field[0] = nb;
    if constexpr (sizeof(T) == 4) {
      if (P->prec == CNPC_PREC_BF16X3) {
        CNPC_TRY(contract_mfma(fields, n3, nb + 1, nb, cc, partial, Cm, s));
      } else {
        CNPC_TRY(contract_mfma_fp<T>(fields, n3, nb + 1, nb, cc, partial, Cm, s));
      }
    } else {
      CNPC_TRY(contract_mfma_fp<T>(fields, n3, nb + 1, nb, cc, partial, Cm, s));
    }
    hipLaunchKernelGGL(k_sugi_accum, dim3((nb * nb + 255) / 256), dim3(256), 0, s, Cm, nb, 2, coef, accum);
    CNPC_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_fill_real<T>), dim3(1024), dim3(256), 0, s, slotOne, n3, T(1));
    CNPC_HIP(hipGetLastError());
    return CNPC_OK;
  };
  const int L = P->L;
  const int sbase = CNPC_NORM_SBARLM + 2 * (L == 0 ? 0 : (L == 2 ? 1 : 4));
  bool noise_pass = false;
  // noise line-of-sight field: scale * [(src / W) N_0^* / W - sgn Sbar C / W^2]
  auto load_los_noise = [&](T* slot, const cx<T>* src, int div, int sidx, double sgn, double scale) -> cnpc_status {
    hipLaunchKernelGGL((k_los_noise<T>), dim3(gb), dim3(256), 0, s, P->desc.n, m, P->desc.assign,
                       P->desc.interlace, div, src, FN0, norms, sidx, sgn, scale, spec);
    CNPC_HIP(hipGetLastError());
    return shell_c2r<T>(&dg, m, spec, P->thr.data(), nb + 1, 0, 1, false, slot, scr, s);
  };
  auto run_pass = [&]() -> cnpc_status {
  int curM = 1;  // no line-of-sight field loaded yet (loaded M are <= 0)
  for (size_t q = 0; q < P->subw.size(); ++q) {
    const int m1 = P->sub[4 * q], m2 = P->sub[4 * q + 1], M = P->sub[4 * q + 2], flag = P->sub[4 * q + 3];
    const double wgt = P->subw[q];
    if (M != curM) {
      // G^M = (-1)^M conj(G^|M|) for M < 0: g = (-1)^M c2r[A/W], h = (-1)^M c2r[B/W]
      const int am = -M;
      const double sg = (am & 1) ? -1.0 : 1.0;
      const cx<T>* A = L == 0 ? F0 : ylm + (am == 0 ? 0 : (int64_t)(2 * am - 1) * bsz);
      if (noise_pass) {
        // P^M = (-1)^M conj(P^|M|) for M < 0, P^|M| = (A - i B)/W N_0^*/W - Sbar C/W^2:
        // g = (-1)^M c2r[A N_0^*/W^2 - Re Sbar C/W^2], h = (-1)^M c2r[B N_0^*/W^2
        // + Im Sbar C/W^2] (Sbar of (L, |M|)); M = 0: g only
        const int si = sbase + 2 * am;
        CNPC_TRY(load_los_noise(slotG, A, L == 0 ? 0 : 1, si, 1.0, am == 0 ? 1.0 : sg));
        if (am > 0) CNPC_TRY(load_los_noise(slotH, ylm + (int64_t)(2 * am) * bsz, 1, si + 1, -1.0, sg));
      } else if (L == 0) {
        // G_0^0 = c2r[F_0]: F_0 is already compensated
        CNPC_TRY(shell_c2r<T>(&dg, m, F0, P->thr.data(), nb + 1, 0, 1, false, slotG, scr, s));
      } else {
        CNPC_TRY(load_los(slotG, A, am == 0 ? 1.0 : sg));
        if (am > 0) CNPC_TRY(load_los(slotH, ylm + (int64_t)(2 * am) * bsz, sg));
      }
      curM = M;
    }
    // the imaginary part b of F_l^m vanishes for even l and m = 0; the real
    // part a for odd l and m = 0 (its contractions then add zero)
    const bool b1 = m1 != 0 || (P->l1 & 1) == 1, b2 = m2 != 0 || (P->l2 & 1) == 1;
    if (flag == 2) {
      // F^m(k1) F^-m(k2) G_L^0 = (-1)^(l+m) [a(k1) a(k2) + b(k1) b(k2)] g
      // (F^-m = (-1)^(l+m) conj(F^m)): one leg's shell fields contracted
      // within the list (symmetric in k1, k2)
      const double sgm = ((P->l1 + m1) & 1) ? -wgt : wgt;
      CNPC_TRY(load_leg(slotP, P->l1, m1, 0));
      CNPC_TRY(contract_self(sgm));
      if (b1) {
        CNPC_TRY(load_leg(slotP, P->l1, m1, 1));
        CNPC_TRY(contract_self(sgm));
      }
      continue;
    }
    const int tr = flag == 1 ? 1 : 0;
    // Re[F1 F2 G] = a1 (a2 g - b2 h) + b1 (-b2 g - a2 h)
    CNPC_TRY(load_leg(slotQa, P->l2, m2, 0));
    if (b2) CNPC_TRY(load_leg(slotQb, P->l2, m2, 1));
    CNPC_TRY(load_leg(slotP, P->l1, m1, 0));
    CNPC_TRY(contract_add(slotQa, slotG, 1.0, (b2 && M != 0) ? slotQb : nullptr, slotH, -1.0, wgt, tr));
    if (b1 && (b2 || M != 0)) {
      CNPC_TRY(load_leg(slotP, P->l1, m1, 1));
      CNPC_TRY(contract_add(b2 ? slotQb : nullptr, slotG, -1.0, M != 0 ? slotQa : nullptr, slotH, -1.0, wgt, tr));
    }
  }
  return CNPC_OK;
  };
  CNPC_TRY(run_pass());
  if (FN0) {
    hipLaunchKernelGGL(k_fill_ones<T>, dim3(256), dim3(256), 0, s, ones, bsz);
    CNPC_HIP(hipGetLastError());
    legsrc = ones;
    accum = acc2;
    noise_pass = true;
    CNPC_TRY(run_pass());
  }
  SugiFin f;
  f.l1 = P->l1;
  f.l2 = P->l2;
  f.L = P->L;
  f.nb = nb;
  f.next = P->next;
  f.hn = P->hn;
  f.n3 = (double)n3;
  f.counts = P->d_counts;
  f.wq3 = P->d_wq3;
  hipLaunchKernelGGL(k_sugi_finalize, dim3((nb * nb + 255) / 256), dim3(256), 0, s, f, acc, FN0 ? acc2 : nullptr,
                     noise, norms, raw, shot, value);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

}  // namespace cnpc

using namespace cnpc;

#include <complex>

// Real decomposition of the tripolar basis (appendix on the real decomposition
// of bipolar and tripolar bases): with X_lm = sum_n V_mn Y_l^n (the real
// harmonics of the spherical-harmonics appendix) and U = V^-1 = V^dagger,
// A^{n1 n2 N} = 1/H sum_{m1 m2 M} U_m1n1 U_m2n2 U_MN (l1 l2 L; m1 m2 M).
static std::complex<double> real_v(int ell, int m, int n) {  // V^l_mn
  const double r2 = 1.0 / std::sqrt(2.0), sg = (std::abs(m) & 1) ? -1.0 : 1.0;
  if (m == 0) return n == 0 ? 1.0 : 0.0;
  if (m < 0) {
    if (n == m) return {0.0, r2};
    if (n == -m) return {0.0, -r2 * sg};
    return 0.0;
  }
  if (n == -m) return r2;
  if (n == m) return r2 * sg;
  return 0.0;
}

extern "C" {

cnpc_status cnpc_tripolar_real_coeffs(int32_t l1, int32_t l2, int32_t L, double* coeffs, int32_t* nonzero) {
  API_BEGIN;
  for (int l : {l1, l2, L}) CNPC_REQUIRE(l >= 0 && l <= 8, "l1, l2, L must be in [0, 8]");
  CNPC_REQUIRE(L >= std::abs(l1 - l2) && L <= l1 + l2 && (l1 + l2 + L) % 2 == 0,
               "(l1, l2, L) must satisfy the triangle rule with an even sum");
  const double H = wigner3j_host(l1, l2, L, 0, 0, 0);
  int nz = 0;
  for (int n1 = -l1; n1 <= l1; ++n1)
    for (int n2 = -l2; n2 <= l2; ++n2)
      for (int N = -L; N <= L; ++N) {
        std::complex<double> a = 0.0;
        for (int m1 = -l1; m1 <= l1; ++m1)
          for (int m2 = -l2; m2 <= l2; ++m2) {
            const int M = -m1 - m2;
            if (std::abs(M) > L) continue;
            const double w = wigner3j_host(l1, l2, L, m1, m2, M);
            if (w == 0.0) continue;
            // U_mn = conj(V_nm)
            a += w * std::conj(real_v(l1, n1, m1)) * std::conj(real_v(l2, n2, m2)) * std::conj(real_v(L, N, M));
          }
        a /= H;
        CNPC_REQUIRE(std::fabs(a.imag()) <= 1e-12, "non-real coefficient (internal error)");
        const double v = std::fabs(a.real()) > 1e-12 ? a.real() : 0.0;
        if (v != 0.0) ++nz;
        if (coeffs) coeffs[((n1 + l1) * (2 * l2 + 1) + (n2 + l2)) * (2 * L + 1) + (N + L)] = v;
      }
  if (nonzero) *nonzero = nz;
  return CNPC_OK;
}

int32_t cnpc_sugi_paired_count(int32_t l1, int32_t l2, int32_t L) {
  if (l1 < 0 || l2 < 0 || L < 0 || l1 > 8 || l2 > 8 || L > 8) return -1;
  int c = 0;
  for (int M = -L; M <= 0; ++M)
    for (int m1 = -l1; m1 <= l1; ++m1) {
      const int m2 = -m1 - M;
      if (std::abs(m2) > l2 || (M == 0 && m1 > 0)) continue;
      if (wigner3j_host(l1, l2, L, m1, m2, M) != 0.0) ++c;
    }
  return c;
}

size_t cnpc_sugi_workspace_size(const cnpc_mesh_desc* d, const cnpc_kbins* b) {
  if (check_desc(d) != CNPC_OK || check_bins(d, b) != CNPC_OK) return 0;
  return sugi_ws_bytes(d, b);
}

cnpc_status cnpc_sugi_plan_create(cnpc_bispec_plan** plan, const cnpc_mesh_desc* d, const cnpc_kbins* b,
                                  int32_t l1, int32_t l2, int32_t L, int32_t prec) {
  API_BEGIN;
  CNPC_REQUIRE(plan != nullptr, "null plan pointer");
  *plan = nullptr;
  CNPC_TRY(check_desc(d));
  CNPC_TRY(check_bins(d, b));
  for (int l : {l1, l2}) CNPC_REQUIRE(l >= 0 && l <= 4, "l1, l2 must be in [0, 4]");
  CNPC_REQUIRE(L == 0 || L == 2 || L == 4, "L must be 0, 2 or 4");
  CNPC_REQUIRE((l1 + l2) % 2 == 0, "l1 + l2 must be even");
  CNPC_REQUIRE(L >= std::abs(l1 - l2) && L <= l1 + l2, "(l1, l2, L) must satisfy the triangle rule");
  CNPC_REQUIRE(prec == CNPC_PREC_F64 || prec == CNPC_PREC_F32 || prec == CNPC_PREC_BF16X3, "unknown precision");
  CNPC_REQUIRE(!(prec == CNPC_PREC_F64 && d->dtype != CNPC_F64), "CNPC_PREC_F64 needs FP64 fields");
  CNPC_REQUIRE(!(prec != CNPC_PREC_F64 && d->dtype != CNPC_F32), "FP32 / split-BF16 contraction needs FP32 fields");
  CNPC_REQUIRE(b->kmin == 0.0, "bispectrum bins must start at k = 0 (closure on bin centres)");
  const double kny = M_PI * d->n / d->boxsize;
  CNPC_REQUIRE((2 * b->nbins - 1) * b->dk <= kny, "the line-of-sight field needs bins up to 2 k_max below Nyquist");
  CNPC_REQUIRE(prec != CNPC_PREC_BF16X3 || b->nbins <= 22, "split-BF16 Sugiyama contraction: at most 22 shells");
  CNPC_REQUIRE(b->nbins <= MAX_COLS, "Sugiyama contraction: at most %d shells", MAX_COLS);
  return sugi_plan_create(plan, d, b, l1, l2, L, prec);
}

cnpc_status cnpc_sugiyama(const cnpc_bispec_plan* p, const void* F0, const void* ylm, const double* noise_means,
                          const double* norms, double* raw, double* shot, double* value, void* ws, size_t ws_bytes,
                          void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr && p->est == CNPC_EST_SUGIYAMA, "need a plan of cnpc_sugi_plan_create");
  CNPC_REQUIRE(F0 && norms && raw && shot && value && ws, "null pointer argument");
  CNPC_REQUIRE(p->L == 0 || ylm != nullptr, "L > 0 needs the Y_L^M spectra of delta");
  if (p->desc.dtype == CNPC_F64)
    return sugi_run_t<double>(p, (const cx<double>*)F0, (const cx<double>*)ylm, nullptr, noise_means, norms, raw,
                              shot, value, ws, ws_bytes, as_stream(stream));
  return sugi_run_t<float>(p, (const cx<float>*)F0, (const cx<float>*)ylm, nullptr, noise_means, norms, raw, shot,
                           value, ws, ws_bytes, as_stream(stream));
}

cnpc_status cnpc_sugiyama_fft_noise(const cnpc_bispec_plan* p, const void* F0, const void* ylm, const void* FN0,
                                    const double* noise_means, const double* norms, double* raw, double* shot,
                                    double* value, void* ws, size_t ws_bytes, void* stream) {
  API_BEGIN;
  CNPC_REQUIRE(p != nullptr && p->est == CNPC_EST_SUGIYAMA, "need a plan of cnpc_sugi_plan_create");
  CNPC_REQUIRE(F0 && FN0 && noise_means && norms && raw && shot && value && ws, "null pointer argument");
  CNPC_REQUIRE(p->L == 0 || ylm != nullptr, "L > 0 needs the Y_L^M spectra of delta");
  if (p->desc.dtype == CNPC_F64)
    return sugi_run_t<double>(p, (const cx<double>*)F0, (const cx<double>*)ylm, (const cx<double>*)FN0,
                              noise_means, norms, raw, shot, value, ws, ws_bytes, as_stream(stream));
  return sugi_run_t<float>(p, (const cx<float>*)F0, (const cx<float>*)ylm, (const cx<float>*)FN0, noise_means,
                           norms, raw, shot, value, ws, ws_bytes, as_stream(stream));
}

}  // extern "C"
