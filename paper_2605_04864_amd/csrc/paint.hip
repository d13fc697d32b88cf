// Catalog sums, normalisations and FKP mass assignment (CIC / TSC, interlacing).
//
// Painting: particles are counting-sorted by 16^3-node tile (LDS-aggregated
// counts, one global atomic per (workgroup, tile)), each tile's particles are
// accumulated into a 19^3-node LDS block (the tile plus the stencil halo) with
// LDS atomics, blocks are written out without atomics, and a fold pass sums
// the <= 8 blocks covering every node while forming delta = n_g - alpha n_r and
// N = n_g(w^2) + alpha^2 n_r(w^2).
#include "paint.h"

namespace cnpc {

constexpr int TILE = 16;
constexpr int BW = TILE + 3;           // block width: nodes c-1 .. c+2 around tile
constexpr int BVOL = BW * BW * BW;     // 6859
constexpr int SORT_BLOCK = 1024;
constexpr int SORT_PER_THREAD = 64;    // particles per thread per sort workgroup
constexpr int LDS_TILES_MAX = 8192;    // LDS-aggregated sort up to this many tiles

// ------------------------------------------------------------ catalog sums --
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_catalog_sums(const uint32_t* __restrict__ pos,
                                                      const float* __restrict__ w, int64_t n,
                                                      SumsArgs a, double* __restrict__ partial) {
  double acc[CNPC_SUMS_LEN];
#pragma unroll
  for (int q = 0; q < CNPC_SUMS_LEN; ++q) acc[q] = 0.0;
  const double scale = a.boxsize / 4294967296.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w ? (double)w[i] : 1.0;
    const double w2 = wi * wi, w3 = w2 * wi;
    acc[0] += wi;
    acc[1] += w2;
    acc[2] += w3;
    double ux, uy, uz;
    if (a.global_los) {
      ux = a.los[0]; uy = a.los[1]; uz = a.los[2];
    } else {
      const double rx = (double)pos[i] * scale - a.obs[0];
      const double ry = (double)pos[n + i] * scale - a.obs[1];
      const double rz = (double)pos[2 * n + i] * scale - a.obs[2];
      const double inv = 1.0 / sqrt(rx * rx + ry * ry + rz * rz);
      ux = rx * inv; uy = ry * inv; uz = rz * inv;
    }
    double re[5], im[5];
    int q = 3;
    // (l, m) order: (0,0), (2,0..2), (4,0..4); accumulate w^3 conj(y_l^m)
    acc[q++] += w3;  // y_0^0 = 1
    acc[q++] += 0.0;
    racah_ylm<double>(2, ux, uy, uz, re, im);
    for (int m = 0; m <= 2; ++m) { acc[q++] += w3 * re[m]; acc[q++] -= w3 * im[m]; }
    racah_ylm<double>(4, ux, uy, uz, re, im);
    for (int m = 0; m <= 4; ++m) { acc[q++] += w3 * re[m]; acc[q++] -= w3 * im[m]; }
  }
  __shared__ double red[4][CNPC_SUMS_LEN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CNPC_SUMS_LEN; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < CNPC_SUMS_LEN) {
    double v = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += red[k][threadIdx.x];
    partial[(int64_t)blockIdx.x * CNPC_SUMS_LEN + threadIdx.x] = v;
  }
}

__global__ void __launch_bounds__(64) k_reduce_partials(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out) {
  // block q sums column q over the partials in a fixed order (deterministic)
  const int q = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 64) v += partial[(int64_t)b * CNPC_SUMS_LEN + q];
  v = wave_sum(v);
  if (threadIdx.x == 0) out[q] = v;
}

__global__ void k_norms(const double* __restrict__ gs, const double* __restrict__ rs, int64_t ngal,
                        double boxsize, double* __restrict__ nm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double alpha = gs[0] / rs[0];
  const double nbar = (double)ngal / (boxsize * boxsize * boxsize);
  const double I22 = alpha * nbar * rs[1];
  const double I33 = alpha * nbar * nbar * rs[2];
  nm[CNPC_NORM_ALPHA] = alpha;
  nm[CNPC_NORM_NBAR] = nbar;
  nm[CNPC_NORM_I22] = I22;
  nm[CNPC_NORM_I33] = I33;
  nm[CNPC_NORM_N0] = (gs[1] + alpha * alpha * rs[1]) / I22;
  nm[CNPC_NORM_SBAR] = gs[2] - alpha * alpha * alpha * rs[2];
  const double a3 = alpha * alpha * alpha;
  for (int q = 0; q < 2 * CNPC_NYLM_SUMS; ++q) nm[CNPC_NORM_SBARLM + q] = gs[3 + q] - a3 * rs[3 + q];
}

// ------------------------------------------------------------------- sort --
__device__ __forceinline__ int tile_of(uint32_t px, uint32_t py, uint32_t pz, int shift, int nt) {
  const int tx = (int)(px >> shift) >> 4, ty = (int)(py >> shift) >> 4, tz = (int)(pz >> shift) >> 4;
  return (tx * nt + ty) * nt + tz;
}

// count[t] += number of particles in tile t (LDS aggregation when it fits)
__global__ void __launch_bounds__(SORT_BLOCK) k_tile_count(const uint32_t* __restrict__ pos, int64_t n,
                                                           int shift, int nt, int ntiles,
                                                           uint32_t* __restrict__ count) {
  extern __shared__ uint32_t lcount[];
  const bool lds = ntiles <= LDS_TILES_MAX;
  const int64_t chunk = (int64_t)SORT_BLOCK * SORT_PER_THREAD;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  if (lds) {
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) lcount[t] = 0;
    __syncthreads();
  }
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int t = tile_of(pos[i], pos[n + i], pos[2 * n + i], shift, nt);
    if (lds) atomicAdd(&lcount[t], 1u);
    else atomicAdd(&count[t], 1u);
  }
  if (lds) {
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
      const uint32_t c = lcount[t];
      if (c) atomicAdd(&count[t], c);
    }
  }
}

// exclusive scan of count -> start, cursor = start (one workgroup)
__global__ void __launch_bounds__(1024) k_tile_scan(const uint32_t* __restrict__ count, int ntiles,
                                                    uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ cursor) {
  __shared__ uint32_t part[1024];
  const int per = (ntiles + 1023) / 1024;
  const int t0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int t = t0; t < min(ntiles, t0 + per); ++t) s += count[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int t = t0; t < min(ntiles, t0 + per); ++t) {
    start[t] = run;
    cursor[t] = run;
    run += count[t];
  }
}

__global__ void __launch_bounds__(SORT_BLOCK) k_tile_scatter(const uint32_t* __restrict__ pos,
                                                             const float* __restrict__ w, int64_t n,
                                                             int shift, int nt, int ntiles,
                                                             uint32_t* __restrict__ cursor,
                                                             uint32_t* __restrict__ spos,
                                                             float* __restrict__ sw) {
  extern __shared__ uint32_t lmem[];
  const bool lds = ntiles <= LDS_TILES_MAX;
  uint32_t* lcount = lmem;
  uint32_t* lbase = lmem + (lds ? ntiles : 0);
  const int64_t chunk = (int64_t)SORT_BLOCK * SORT_PER_THREAD;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  if (lds) {
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) lcount[t] = 0;
    __syncthreads();
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
      atomicAdd(&lcount[tile_of(pos[i], pos[n + i], pos[2 * n + i], shift, nt)], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
      const uint32_t c = lcount[t];
      lbase[t] = c ? atomicAdd(&cursor[t], c) : 0u;
      lcount[t] = 0;
    }
    __syncthreads();
  }
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const uint32_t px = pos[i], py = pos[n + i], pz = pos[2 * n + i];
    const int t = tile_of(px, py, pz, shift, nt);
    const uint32_t slot = lds ? lbase[t] + atomicAdd(&lcount[t], 1u) : atomicAdd(&cursor[t], 1u);
    spos[slot] = px;
    spos[n + slot] = py;
    spos[2 * n + slot] = pz;
    if (w) sw[slot] = w[i];
  }
}

// ------------------------------------------------------------------ paint --
// 1-D stencil: node offsets relative to the base cell c = floor(u) and weights.
template <typename T>
__device__ __forceinline__ int stencil_1d(uint32_t p, int shift, int assign, int phase, T* wt) {
  const uint32_t mask = (shift >= 32) ? 0xffffffffu : ((1u << shift) - 1u);
  const int64_t f = (int64_t)(p & mask);
  const int64_t one = (int64_t)1 << shift, half = one >> 1;
  const T inv = T(1) / T(one);
  if (assign == CNPC_TSC) {
    // phase A: i = floor(u + 1/2); phase B: i = floor(u) (u - 1/2 + 1/2)
    int off;
    int64_t dfix;
    if (phase == 0) {
      if (f >= half) { off = 1; dfix = f - one; } else { off = 0; dfix = f; }
    } else {
      off = 0;
      dfix = f - half;
    }
    const T d = T(dfix) * inv;
    const T a = T(0.5) - d, b = T(0.5) + d;
    wt[0] = T(0.5) * a * a;
    wt[1] = T(0.75) - d * d;
    wt[2] = T(0.5) * b * b;
    return off - 1;  // first node offset
  }
  // CIC: phase A: nodes c, c+1 with d = frac; phase B: u - 1/2
  if (phase == 0) {
    const T d = T(f) * inv;
    wt[0] = T(1) - d;
    wt[1] = d;
    return 0;
  }
  int off;
  int64_t dfix;
  if (f >= half) { off = 0; dfix = f - half; } else { off = -1; dfix = f + half; }
  const T d = T(dfix) * inv;
  wt[0] = T(1) - d;
  wt[1] = d;
  return off;
}

// Contributions are accumulated as 64-bit fixed point (2^-40 units) with
// integer LDS atomics: on gfx950 integer LDS atomics run at full rate while
// FP32 LDS atomics are an order of magnitude slower, and integer sums do not
// depend on the order in which the threads add (bit-reproducible blocks).
constexpr double FIX_SCALE = 1099511627776.0;  // 2^40
constexpr double FIX_INV = 1.0 / 1099511627776.0;

template <typename T, int ASSIGN>
__global__ void __launch_bounds__(512) k_paint_tiles(const uint32_t* __restrict__ spos,
                                                     const float* __restrict__ sw, int64_t n,
                                                     const uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ count, int shift,
                                                     int nphase, int ph0, int nph, int power,
                                                     T* __restrict__ blocks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem_raw);  // [nph][BVOL]
  const int t = blockIdx.x;
  for (int i = threadIdx.x; i < nph * BVOL; i += blockDim.x) acc[i] = 0ull;
  __syncthreads();
  const uint32_t s0 = start[t], cnt = count[t];
  constexpr int NP = ASSIGN == CNPC_TSC ? 3 : 2;
  for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int64_t i = (int64_t)s0 + k;
    const uint32_t px = spos[i], py = spos[n + i], pz = spos[2 * n + i];
    T wv = T(1);
    if (sw) {
      wv = T(sw[i]);
      if (power == 2) wv *= wv;
    }
    const int bx = ((int)(px >> shift) & 15) + 1;
    const int by = ((int)(py >> shift) & 15) + 1;
    const int bz = ((int)(pz >> shift) & 15) + 1;
    for (int q = 0; q < nph; ++q) {
      const int ph = ph0 + q;
      T wx[3], wy[3], wz[3];
      const int ox = stencil_1d<T>(px, shift, ASSIGN, ph, wx);
      const int oy = stencil_1d<T>(py, shift, ASSIGN, ph, wy);
      const int oz = stencil_1d<T>(pz, shift, ASSIGN, ph, wz);
      unsigned long long* a =
          acc + q * BVOL + (bx + ox) * BW * BW + (by + oy) * BW + (bz + oz);
#pragma unroll
      for (int ix = 0; ix < NP; ++ix) {
        const T vx = wv * wx[ix];
#pragma unroll
        for (int iy = 0; iy < NP; ++iy) {
          const T vxy = vx * wy[iy];
#pragma unroll
          for (int iz = 0; iz < NP; ++iz) {
            const long long fixv = __double2ll_rn((double)(vxy * wz[iz]) * FIX_SCALE);
            atomicAdd(&a[ix * BW * BW + iy * BW + iz], (unsigned long long)fixv);
          }
        }
      }
    }
  }
  __syncthreads();
  T* out = blocks + ((int64_t)t * nphase + ph0) * BVOL;
  for (int i = threadIdx.x; i < nph * BVOL; i += blockDim.x)
    out[i] = T((double)(long long)acc[i] * FIX_INV);
}

// sum of the blocks of set `s` covering node (x, y, z), phase ph
template <typename T>
__device__ __forceinline__ T gather_node(const T* __restrict__ blocks, int nt, int nphase, int ph,
                                         int x, int y, int z) {
  int tx[2], lx[2], nx = 0, ty[2], ly[2], ny = 0, tz[2], lz[2], nz = 0;
  auto cover = [nt](int c, int* tt, int* ll, int& k) {
    const int t = c >> 4, r = c & 15;
    tt[k] = t; ll[k] = r + 1; ++k;
    if (r <= 1) { tt[k] = (t - 1 + nt) % nt; ll[k] = r + 17; ++k; }
    else if (r == 15) { tt[k] = (t + 1) % nt; ll[k] = 0; ++k; }
  };
  cover(x, tx, lx, nx);
  cover(y, ty, ly, ny);
  cover(z, tz, lz, nz);
  T v = T(0);
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nz; ++c) {
        const int64_t tile = ((int64_t)tx[a] * nt + ty[b]) * nt + tz[c];
        v += blocks[(tile * nphase + ph) * BVOL + (lx[a] * BW + ly[b]) * BW + lz[c]];
      }
  return v;
}

// out_delta = sum_s cd[s] blocks_s, out_noise = sum_s cn[s] blocks_s; coefficients
// come from alpha on the device: sets (g, r) for unit weights, (g w, r w, g w^2,
// r w^2) for weighted catalogs.
template <typename T>
__global__ void __launch_bounds__(256) k_fold(FoldArgs<T> fa, const double* __restrict__ norms,
                                              T* __restrict__ delta, T* __restrict__ noise) {
  const int n = fa.n;
  const int64_t n3 = (int64_t)n * n * n;
  const double alpha = norms[CNPC_NORM_ALPHA];
  double cd[4], cn[4];
  if (fa.nsets == 2) {
    cd[0] = 1.0; cd[1] = -alpha; cn[0] = 1.0; cn[1] = alpha * alpha;
  } else {
    cd[0] = 1.0; cd[1] = -alpha; cd[2] = 0.0; cd[3] = 0.0;
    cn[0] = 0.0; cn[1] = 0.0; cn[2] = 1.0; cn[3] = alpha * alpha;
  }
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n3 * fa.nphase;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int ph = (int)(idx / n3);
    const int64_t cell = idx - ph * n3;
    const int z = (int)(cell % n), y = (int)((cell / n) % n), x = (int)(cell / ((int64_t)n * n));
    T d = T(0), q = T(0);
    for (int s = 0; s < fa.nsets; ++s) {
      const T v = gather_node<T>(fa.blocks[s], fa.nt, fa.nphase, ph, x, y, z);
      d += T(cd[s]) * v;
      q += T(cn[s]) * v;
    }
    delta[idx] = d;
    if (noise) noise[idx] = q;
  }
}

// ------------------------------------------------------------------- host --
cnpc_status launch_catalog_sums(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w,
                                int64_t n, double* sums, void* ws, size_t ws_bytes,
                                hipStream_t s) {
  const int nblocks = 1024;
  if (ws_bytes < (size_t)nblocks * CNPC_SUMS_LEN * sizeof(double)) {
    set_error("catalog_sums workspace too small");
    return CNPC_EWORKSPACE;
  }
  SumsArgs a;
  a.boxsize = d->boxsize;
  for (int i = 0; i < 3; ++i) { a.obs[i] = d->observer[i]; a.los[i] = d->los[i]; }
  a.global_los = d->los_mode == CNPC_LOS_GLOBAL;
  double* partial = reinterpret_cast<double*>(ws);
  kt_begin(CNPC_KT_SUMS, s);
  hipLaunchKernelGGL(k_catalog_sums, dim3(nblocks), dim3(256), 0, s, pos, w, n, a, partial);
  kt_end(CNPC_KT_SUMS, s);
  CNPC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_partials, dim3(CNPC_SUMS_LEN), dim3(64), 0, s, partial, nblocks, sums);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_norms(const cnpc_mesh_desc* d, const double* gs, const double* rs, int64_t ngal,
                         double* norms, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(64), 0, s, gs, rs, ngal, d->boxsize, norms);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

PaintLayout paint_layout(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, bool weighted) {
  PaintLayout L;
  const int nt = d->n / TILE;
  L.nt = nt;
  L.ntiles = nt * nt * nt;
  L.nphase = d->interlace ? 2 : 1;
  L.nsets = weighted ? 4 : 2;
  const size_t es = esize(d->dtype);
  size_t off = 0;
  for (int c = 0; c < 2; ++c) {
    const int64_t np = c == 0 ? ngal : nran;
    L.off_spos[c] = off; off = align_up(off + (size_t)np * 3 * 4);
    L.off_sw[c] = off; off = align_up(off + (weighted ? (size_t)np * 4 : 0));
    L.off_count[c] = off; off = align_up(off + (size_t)L.ntiles * 4);
    L.off_start[c] = off; off = align_up(off + (size_t)L.ntiles * 4);
    L.off_cursor[c] = off; off = align_up(off + (size_t)L.ntiles * 4);
  }
  for (int k = 0; k < L.nsets; ++k) {
    L.off_blocks[k] = off;
    off = align_up(off + (size_t)L.ntiles * L.nphase * BVOL * es);
  }
  L.total = off;
  return L;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <typename T>
static cnpc_status paint_t(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                           int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                           const double* norms, T* delta, T* noise, unsigned char* ws,
                           const PaintLayout& L, hipStream_t s) {
  const int shift = 32 - ilog2_host(d->n);
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  const uint32_t* cpos[2] = {gpos, rpos};
  const float* cw[2] = {gw, rw};
  const int64_t cn[2] = {ngal, nran};
  const size_t lds_sort = L.ntiles <= LDS_TILES_MAX ? (size_t)L.ntiles * 4 : 0;
  const size_t lds_scatter = L.ntiles <= LDS_TILES_MAX ? (size_t)L.ntiles * 8 : 0;
  // phases per launch so that the 64-bit LDS blocks fit the workgroup limit
  const int nph = ((size_t)L.nphase * BVOL * 8 <= lds_limit()) ? L.nphase : 1;
  const size_t lds_paint = (size_t)nph * BVOL * 8;
  FoldArgs<T> fa;
  fa.n = d->n;
  fa.nt = L.nt;
  fa.nphase = L.nphase;
  fa.nsets = L.nsets;
  for (int c = 0; c < 2; ++c) {
    const int64_t n = cn[c];
    uint32_t* count = reinterpret_cast<uint32_t*>(ws + L.off_count[c]);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.off_start[c]);
    uint32_t* cursor = reinterpret_cast<uint32_t*>(ws + L.off_cursor[c]);
    uint32_t* spos = reinterpret_cast<uint32_t*>(ws + L.off_spos[c]);
    float* sw = cw[c] ? reinterpret_cast<float*>(ws + L.off_sw[c]) : nullptr;
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count, (int64_t)L.ntiles);
    CNPC_HIP(hipGetLastError());
    const int64_t chunk = (int64_t)SORT_BLOCK * SORT_PER_THREAD;
    const int64_t nblk = (n + chunk - 1) / chunk;
    if (nblk > 0) {
      kt_begin(CNPC_KT_SORT, s);
      hipLaunchKernelGGL(k_tile_count, dim3((unsigned)nblk), dim3(SORT_BLOCK), lds_sort, s, cpos[c], n,
                         shift, L.nt, L.ntiles, count);
      kt_end(CNPC_KT_SORT, s);
      CNPC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, count, L.ntiles, start, cursor);
    CNPC_HIP(hipGetLastError());
    if (nblk > 0) {
      kt_begin(CNPC_KT_SORT, s);
      hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)nblk), dim3(SORT_BLOCK), lds_scatter, s,
                         cpos[c], cw[c], n, shift, L.nt, L.ntiles, cursor, spos, sw);
      kt_end(CNPC_KT_SORT, s);
      CNPC_HIP(hipGetLastError());
    }
    const int npow = weighted ? 2 : 1;
    for (int pw = 0; pw < npow; ++pw) {
      const int set = weighted ? (pw * 2 + c) : c;
      T* blocks = reinterpret_cast<T*>(ws + L.off_blocks[set]);
      for (int ph0 = 0; ph0 < L.nphase; ph0 += nph) {
        kt_begin(CNPC_KT_PAINT, s);
        if (d->assign == CNPC_TSC)
          hipLaunchKernelGGL((k_paint_tiles<T, CNPC_TSC>), dim3(L.ntiles), dim3(512), lds_paint, s, spos,
                             sw, n, start, count, shift, L.nphase, ph0, nph, pw + 1, blocks);
        else
          hipLaunchKernelGGL((k_paint_tiles<T, CNPC_CIC>), dim3(L.ntiles), dim3(512), lds_paint, s, spos,
                             sw, n, start, count, shift, L.nphase, ph0, nph, pw + 1, blocks);
        kt_end(CNPC_KT_PAINT, s);
        CNPC_HIP(hipGetLastError());
      }
      fa.blocks[set] = blocks;
    }
  }
  const int64_t total = (int64_t)d->n * d->n * d->n * L.nphase;
  const int64_t nb = std::min<int64_t>((total + 255) / 256, 65536);
  kt_begin(CNPC_KT_FOLD, s);
  hipLaunchKernelGGL((k_fold<T>), dim3((unsigned)nb), dim3(256), 0, s, fa, norms, delta, noise);
  kt_end(CNPC_KT_FOLD, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_paint(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                         int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                         const double* norms, void* delta, void* noise, void* ws, size_t ws_bytes,
                         hipStream_t s) {
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  PaintLayout L = paint_layout(d, ngal, nran, weighted);
  if (ws_bytes < L.total) {
    set_error("paint workspace too small: need %zu bytes, got %zu", L.total, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (d->dtype == CNPC_F64)
    return paint_t<double>(d, gpos, gw, ngal, rpos, rw, nran, norms, (double*)delta, (double*)noise, w,
                           L, s);
  return paint_t<float>(d, gpos, gw, ngal, rpos, rw, nran, norms, (float*)delta, (float*)noise, w, L,
                        s);
}

}  // namespace cnpc
