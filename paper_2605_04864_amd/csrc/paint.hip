// Catalog sums, normalisations and FKP mass assignment (CIC / TSC, interlacing).
//
// Painting: particles are counting-sorted by 16^3-node tile (two LDS-staged
// steps: by bucket of tiles, then by tile; for the FP32 painter on meshes of
// 256^3 and more the records are 8-byte tile-relative ones from the first step
// on, with a 16-bit tile index beside them up to 2^16 tiles), each tile's
// particles are
// accumulated into a 19^3-node LDS block (the tile plus the stencil halo) with
// LDS atomics, blocks are written out without atomics, and a fold pass sums
// the <= 8 blocks covering every node while forming delta = n_g - alpha n_r and
// N = n_g(w^2) + alpha^2 n_r(w^2).
#include "fft.h"
#include "paint.h"

namespace cnpc {

constexpr int TILE = 16;
constexpr int BW = TILE + 3;           // block width: nodes c-1 .. c+2 around tile
constexpr int BVOL = BW * BW * BW;     // 6859
constexpr int BSTRIDE = 6880;          // elements per (tile, phase) block: BVOL rounded to 32

// Layout of a block (LDS accumulator and memory).  Local node l = 0..18 along
// an axis is node 16 t - 1 + l of the mesh: l = 1..16 are the tile's own
// nodes, l = 17..18 nodes 0..1 of the upper neighbour, l = 0 node 15 of the
// lower one.  Rows (lx, ly) of 19 nodes are stored in row-major order, and
// within a row node lz sits at (lz + 18) mod 19: the 16 own nodes first, then
// the two of the upper neighbour, then the one of the lower neighbour.  So a
// fold reads every row as one run of 16 own values and short runs for the z
// neighbours, and the stencil addresses of a particle stay affine except for
// a node l = 0, which moves to the end of its row.
constexpr int SORT_BLOCK = 1024;
constexpr int SORT_PER_THREAD = 64;    // particles per thread per sort workgroup
constexpr int LDS_TILES_MAX = 8192;    // LDS-aggregated sort up to this many tiles

// ------------------------------------------------------------ tile keys --
struct TileGeom {
  int shift;  // 32 - log2(n): node index = p >> shift
  int nt;     // tiles per side
  int ls;     // log2(S)
  int lnb;    // log2(buckets per side)
};

template <int RS>
struct Rec {
  uint32_t v[RS];
};

// Tile-sorted record of the FP32 painter (unweighted catalogs, meshes of 256^3
// and more): the 21 bits of each coordinate below the tile index, i.e. the 4
// node bits inside the 16-node tile and the top 17 fraction bits, in 8 bytes
// (x | y << 21 | z << 42).  Positions keep a 2^-17 cell grid, finer than FP32
// coordinates of a 256-cell box resolve; needs shift >= 17 (meshes up to 2^15
// per side).  The grid's jitter scales with the cell size, so coarser meshes,
// whose binned k reach closer to their Nyquist wavenumber, keep full records.
__host__ __device__ constexpr bool packs_records(bool f32, int rs, int shift) {
  return f32 && rs == 3 && shift <= 24;
}
__device__ __forceinline__ uint64_t pack_rec(const Rec<3>& r, int shift) {
  const uint32_t m = shift + 4 >= 32 ? 0xffffffffu : ((1u << (shift + 4)) - 1u);
  const int down = shift - 17;
  return (uint64_t)((r.v[0] & m) >> down) | ((uint64_t)((r.v[1] & m) >> down) << 21) |
         ((uint64_t)((r.v[2] & m) >> down) << 42);
}

// a tile-sorted record out: in full, or packed (pack_rec) for the FP32 painter
template <int RS>
__device__ __forceinline__ void put_rec(Rec<RS>* out, uint32_t o, const Rec<RS>& r, bool pack, int shift) {
  if constexpr (RS == 3) {
    if (pack) {
      reinterpret_cast<uint64_t*>(out)[o] = pack_rec(r, shift);
      return;
    }
  }
  out[o] = r;
}

// catalog positions read once by the sums pass: non-temporal loads
__device__ __forceinline__ uint32_t ld_stream(const uint32_t* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ int key_of(int tx, int ty, int tz, const TileGeom& g) {
  const int m = (1 << g.ls) - 1;
  const int b = ((((tx >> g.ls) << g.lnb) | (ty >> g.ls)) << g.lnb) | (tz >> g.ls);
  const int l = ((((tx & m) << g.ls) | (ty & m)) << g.ls) | (tz & m);
  return (b << (3 * g.ls)) | l;
}

__device__ __forceinline__ int tile_key(uint32_t px, uint32_t py, uint32_t pz, const TileGeom& g) {
  return key_of((int)(px >> g.shift) >> 4, (int)(py >> g.shift) >> 4, (int)(pz >> g.shift) >> 4, g);
}

struct CountArgs {
  TileGeom g;
  int ntiles;
  uint32_t* count;  // nullptr: sums only
};

// ------------------------------------------------------------ catalog sums --
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

constexpr int SUMS_THREADS = 1024;
constexpr int SUMS_BLOCKS = 256;

// adds the catalog sums of one particle (weight wi) to acc
template <int LMAX>
__device__ __forceinline__ void sums_add(double* acc, uint32_t px, uint32_t py, uint32_t pz, double wi,
                                       double scale, const SumsArgs& a) {
  const double w2 = wi * wi, w3 = w2 * wi;
  acc[0] += wi;
  acc[1] += w2;
  acc[2] += w3;
  int q = 3;
  // (l, m) order: (0,0), (2,0..2), (4,0..4); accumulate w^3 conj(y_l^m)
  acc[q++] += w3;  // y_0^0 = 1
  acc[q++] += 0.0;
  if constexpr (LMAX < 2) return;
  if (a.global_los) {
    double re[5], im[5];
    racah_ylm<double>(2, a.los[0], a.los[1], a.los[2], re, im);
    for (int m = 0; m <= 2; ++m) { acc[q++] += w3 * re[m]; acc[q++] -= w3 * im[m]; }
    if constexpr (LMAX < 4) return;
    racah_ylm<double>(4, a.los[0], a.los[1], a.los[2], re, im);
    for (int m = 0; m <= 4; ++m) { acc[q++] += w3 * re[m]; acc[q++] -= w3 * im[m]; }
  } else {
    // solid harmonics: y_l^m(r / R) = Q_lm(r_z, R^2) (r_x + i r_y)^m / R^l,
    // the Q_lm of solid_coef written out for l = 2, 4
    const double rx = (double)px * scale - a.obs[0];
    const double ry = (double)py * scale - a.obs[1];
    const double rz = (double)pz * scale - a.obs[2];
    const double z2 = rz * rz;
    const double r2 = rx * rx + ry * ry + z2;
    const double i2 = 1.0 / r2;
    const double c2 = w3 * i2, c4 = c2 * i2;
    const double s2r = rx * rx - ry * ry, s2i = 2.0 * rx * ry;
    const double s3r = s2r * rx - s2i * ry, s3i = s2r * ry + s2i * rx;
    const double s4r = s2r * s2r - s2i * s2i, s4i = 2.0 * s2r * s2i;
    const double q20 = c2 * (1.5 * z2 - 0.5 * r2);
    const double q21 = c2 * -1.22474487139158904910 * rz;
    const double q22 = c2 * 0.61237243569579452455;
    acc[5] += q20;
    acc[7] += q21 * rx; acc[8] -= q21 * ry;
    acc[9] += q22 * s2r; acc[10] -= q22 * s2i;
    if constexpr (LMAX < 4) return;
    const double q40 = c4 * ((4.375 * z2 - 3.75 * r2) * z2 + 0.375 * r2 * r2);
    const double q41 = c4 * rz * (-3.91311896062463196870 * z2 + 1.67705098312484227230 * r2);
    const double q42 = c4 * (2.76699295264733191550 * z2 - 0.39528470752104741650 * r2);
    const double q43 = c4 * -1.47901994577490951707 * rz;
    const double q44 = c4 * 0.52291251658379721749;
    acc[11] += q40;
    acc[13] += q41 * rx; acc[14] -= q41 * ry;
    acc[15] += q42 * s2r; acc[16] -= q42 * s2i;
    acc[17] += q43 * s3r; acc[18] -= q43 * s3i;
    acc[19] += q44 * s4r; acc[20] -= q44 * s4i;
  }
}

// LMAX: Y_lm sums for l <= LMAX (0, 2 or 4); the others stay zero
template <int LMAX>
__global__ void __launch_bounds__(SUMS_THREADS) k_catalog_sums(const uint32_t* __restrict__ pos,
                                                      const float* __restrict__ w, int64_t n,
                                                      SumsArgs a, double* __restrict__ partial,
                                                      CountArgs ca) {
  extern __shared__ uint32_t lcount[];
  const bool count = ca.count != nullptr;
  const bool lds = count && ca.ntiles <= LDS_TILES_MAX;
  if (lds) {
    for (int t = threadIdx.x; t < ca.ntiles; t += blockDim.x) lcount[t] = 0;
    __syncthreads();
  }
  double acc[CNPC_SUMS_LEN];
#pragma unroll
  for (int q = 0; q < CNPC_SUMS_LEN; ++q) acc[q] = 0.0;
  const double scale = a.boxsize / 4294967296.0;
  // U particles per thread and trip: all their loads are issued before any of
  // them is used (fewer for the larger register sets of l > 0)
  constexpr int U = LMAX == 0 ? 4 : (LMAX == 2 ? 2 : 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n; i0 += U * stride) {
    uint32_t px[U], py[U], pz[U];
    float wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      px[u] = py[u] = pz[u] = 0u;
      wv[u] = 1.0f;
      if (i < n) {
        px[u] = ld_stream(pos + i);
        py[u] = ld_stream(pos + n + i);
        pz[u] = ld_stream(pos + 2 * n + i);
        if (w) wv[u] = w[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * stride >= n) break;
      if (count) {
        const int t = tile_key(px[u], py[u], pz[u], ca.g);
        if (lds) atomicAdd(&lcount[t], 1u);
        else atomicAdd(&ca.count[t], 1u);
      }
      sums_add<LMAX>(acc, px[u], py[u], pz[u], (double)wv[u], scale, a);
    }
  }
  __shared__ double red[SUMS_THREADS / 64][CNPC_SUMS_LEN];
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
  if (lds) {
    for (int t = threadIdx.x; t < ca.ntiles; t += blockDim.x) {
      const uint32_t c = lcount[t];
      if (c) atomicAdd(&ca.count[t], c);
    }
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
// Tiles are numbered bucket-major: a bucket is a cube of S^3 tiles (S = min(4,
// nt)), key = bucket * S^3 + tile-in-bucket.  The particles of a catalog are
// moved twice, each time by a counting sort whose workgroups stage their chunk
// in LDS ordered by key and then store it in per-key runs: first by bucket
// (few keys, long runs), then by tile inside the bucket.  Records are AoS:
// (px, py, pz) or (px, py, pz, w bits).
// count[key] += number of particles in the tile (LDS aggregation when it fits)
__global__ void __launch_bounds__(SORT_BLOCK) k_tile_count(const uint32_t* __restrict__ pos, int64_t n,
                                                           TileGeom g, int ntiles,
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
    const int t = tile_key(pos[i], pos[n + i], pos[2 * n + i], g);
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

// Exclusive scan of R values by a workgroup of NT threads: emit(r, sum_{q < r}
// in[q]) for every r, each thread handling a run of consecutive r.  Wave
// prefix sums plus one LDS slot per wave (wsum, NT / 64 entries).
template <int NT, typename Emit>
__device__ void block_exclusive_scan(const uint32_t* in, int R, uint32_t* wsum, Emit emit) {
  const int per = (R + NT - 1) / NT;
  const int t0 = threadIdx.x * per, t1 = min(R, t0 + per);
  uint32_t s = 0;
  for (int t = t0; t < t1; ++t) s += in[t];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t v = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) wsum[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < NT / 64; ++k) {
      const uint32_t c = wsum[k];
      wsum[k] = run;
      run += c;
    }
  }
  __syncthreads();
  uint32_t run = wsum[wv] + v - s;
  for (int t = t0; t < t1; ++t) {
    emit(t, run);
    run += in[t];
  }
}

// start[key] = exclusive scan of count, cursor = start, bucket cursor
// bcur[b] = start[b * S^3] (one workgroup)
__global__ void __launch_bounds__(1024) k_tile_scan(const uint32_t* __restrict__ count, int ntiles,
                                                    int per_bucket, uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ bcur) {
  __shared__ uint32_t wsum[16];
  block_exclusive_scan<1024>(count, ntiles, wsum, [&](int t, uint32_t v) {
    start[t] = v;
    cursor[t] = v;
    if (t % per_bucket == 0) bcur[t / per_bucket] = v;
  });
}

// k_tile_scan (workgroup 0) and, in workgroups 1 .. CNPC_SUMS_LEN, the
// fixed-order column sums of k_reduce_partials (first wavefront): the two
// steps between the first and the second sort step of a fused sort, one launch.
__global__ void __launch_bounds__(1024) k_tile_scan_sums(const uint32_t* __restrict__ count, int ntiles,
                                                         int per_bucket, uint32_t* __restrict__ start,
                                                         uint32_t* __restrict__ cursor, uint32_t* __restrict__ bcur,
                                                         const double* __restrict__ partial, int nblocks,
                                                         double* __restrict__ sums) {
  __shared__ uint32_t wsum[16];
  if (blockIdx.x == 0) {
    block_exclusive_scan<1024>(count, ntiles, wsum, [&](int t, uint32_t v) {
      start[t] = v;
      cursor[t] = v;
      if (t % per_bucket == 0) bcur[t / per_bucket] = v;
    });
    return;
  }
  if (threadIdx.x >= 64) return;
  const int q = blockIdx.x - 1;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 64) v += partial[(int64_t)b * CNPC_SUMS_LEN + q];
  v = wave_sum(v);
  if (threadIdx.x == 0) sums[q] = v;
}

// zeroes p[0, n) and q[0, m) in one launch
__global__ void k_zero2_u32(uint32_t* p, int64_t n, uint32_t* q, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + m; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n) p[i] = 0u;
    else q[i - n] = 0u;
  }
}

// Size in bytes of the LDS layout of k_partition with nt threads.
__host__ __device__ constexpr size_t partition_lds(int per, int rs, int rcap, int nt) {
  return (size_t)nt * per * (rs * 4 + 2) + (size_t)3 * rcap * 4 + 64;
}

// One counting-sort step over a chunk of NT * PER particles.
// SOA: input is the catalog (pos [3][n], optional w), else records.
// FINE == false: key = bucket (rcap = number of buckets).
// FINE == true, SOA: key = tile key (rcap = number of tiles, one bucket).
// FINE == true, records in bucket order: key = tile key; the chunk's keys lie
// in [bucket(first) S^3, (bucket(last) + 1) S^3); if that range is wider than
// rcap the chunk takes one global atomic per particle instead.
// cursor[key] hands out output slots (initialised to the key's start).
template <bool SOA, bool FINE, int RS, int PER, int NT>
__global__ void __launch_bounds__(NT) k_partition(const uint32_t* __restrict__ pos,
                                                            const float* __restrict__ w,
                                                            const Rec<RS>* __restrict__ rin,
                                                            int64_t n, TileGeom g, int rcap,
                                                            uint32_t* __restrict__ cursor,
                                                            Rec<RS>* __restrict__ rout, bool pack) {
  constexpr int CH = NT * PER;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Rec<RS>* stage = reinterpret_cast<Rec<RS>*>(smem_raw);                        // [CH]
  uint16_t* skey = reinterpret_cast<uint16_t*>(smem_raw + (size_t)CH * RS * 4);  // [CH]
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem_raw + (size_t)CH * (RS * 4 + 2));
  uint32_t* lstart = hist + rcap;
  uint32_t* gbase = lstart + rcap;
  uint32_t* wsum = gbase + rcap;  // 16 slots
  const int64_t c0 = (int64_t)blockIdx.x * CH;
  const int bshift = 3 * g.ls;
  int klo = 0, R;
  if (FINE && !SOA) {
    const Rec<RS> a = rin[c0], b = rin[min(n, c0 + CH) - 1];
    const int kb0 = tile_key(a.v[0], a.v[1], a.v[2], g) >> bshift;
    const int kb1 = tile_key(b.v[0], b.v[1], b.v[2], g) >> bshift;
    klo = kb0 << bshift;
    R = (kb1 - kb0 + 1) << bshift;
  } else {
    R = rcap;
  }
  Rec<RS> r[PER];
  int key[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = c0 + (int64_t)k * NT + threadIdx.x;
    key[k] = -1;
    if (i < n) {
      if (!SOA) {
        r[k] = rin[i];
      } else {
        r[k].v[0] = pos[i];
        r[k].v[1] = pos[n + i];
        r[k].v[2] = pos[2 * n + i];
        if constexpr (RS == 4) r[k].v[3] = __float_as_uint(w[i]);
      }
      const int t = tile_key(r[k].v[0], r[k].v[1], r[k].v[2], g);
      key[k] = FINE ? t - klo : (t >> bshift);
    }
  }
  if (FINE && !SOA && R > rcap) {
    // wide key range: one global slot per particle
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (key[k] >= 0) put_rec(rout, atomicAdd(&cursor[klo + key[k]], 1u), r[k], FINE && pack, g.shift);
    return;
  }
  for (int t = threadIdx.x; t < R; t += NT) hist[t] = 0u;
  __syncthreads();
  uint32_t rank[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) rank[k] = atomicAdd(&hist[key[k]], 1u);
  __syncthreads();
  block_exclusive_scan<NT>(hist, R, wsum, [&](int t, uint32_t v) {
    lstart[t] = v;
    const uint32_t c = hist[t];
    gbase[t] = c ? atomicAdd(&cursor[klo + t], c) : 0u;
  });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) {
      const uint32_t slot = lstart[key[k]] + rank[k];
      stage[slot] = r[k];
      skey[slot] = (uint16_t)key[k];
    }
  __syncthreads();
  const int cnt = (int)min((int64_t)CH, n - c0);
  for (int j = threadIdx.x; j < cnt; j += NT) {
    const int kk = skey[j];
    put_rec(rout, gbase[kk] + (j - lstart[kk]), stage[j], FINE && pack, g.shift);
  }
}

// ------------------------------------------------------ fused bucket pass --
// One read of a catalog does the FP64 catalog sums, the tile histogram and the
// first counting-sort step.  Buckets have a fixed capacity `cap` (bucket b at
// region + b cap): a workgroup reserves its run in bucket b with one atomic on
// bcnt[b] and sends whatever would pass the capacity to the overflow region
// (reserved on *ovf), which the tile pass takes as chunks of mixed buckets.
// Persistent workgroups walk chunks of NT * PER particles, so the LDS tile
// histogram is flushed with one atomic per non-empty tile per workgroup.  With
// `pack` (FP32 painter, unweighted, 256^3 and more, at most 2^16 tiles) a
// record goes out as pack_rec in 8 bytes and its tile index in 2 more, in an
// array after the 8-byte records of its region (both fit the 12-byte records'
// room); the LDS then also stages each record's tile index after the tile
// histogram.
struct BucketArgs {
  TileGeom g;
  int ntiles, nbuckets;
  uint32_t cap;       // records per bucket region
  uint32_t* bcnt;     // [nbuckets] reservations per bucket (may exceed cap)
  uint32_t* ovf;      // overflow records reserved
  uint32_t* tcount;   // [ntiles] tile histogram
  double* partial;    // [gridDim.x][CNPC_SUMS_LEN] catalog-sum partials
  bool pack;          // records out as pack_rec + a 16-bit tile index (rkey / okey)
  uint16_t* rkey;     // [nbuckets * cap] tile index of each region record (pack)
  uint16_t* okey;     // [n] tile index of each overflow record (pack)
};

// LDS bytes of k_bucket_pass
__host__ __device__ constexpr size_t bucket_pass_lds(int per, int rs, int nbuckets, int nt, int ltiles) {
  return (size_t)nt * per * (rs * 4 + 2) + (size_t)6 * nbuckets * 4 + 64 + (size_t)ltiles * 4;
}

// PF: the next chunk's particles are loaded while the current one is sorted
template <int RS, int PER, int NT, int LMAX, bool PF>
__global__ void __launch_bounds__(NT) k_bucket_pass(const uint32_t* __restrict__ pos, const float* __restrict__ w,
                                                    int64_t n, SumsArgs sa, BucketArgs ba,
                                                    Rec<RS>* __restrict__ region, Rec<RS>* __restrict__ ovf_out) {
  constexpr int CH = NT * PER;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Rec<RS>* stage = reinterpret_cast<Rec<RS>*>(smem_raw);                        // [CH]
  uint16_t* skey = reinterpret_cast<uint16_t*>(smem_raw + (size_t)CH * RS * 4);  // [CH]
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem_raw + (size_t)CH * (RS * 4 + 2));
  uint32_t* lstart = hist + ba.nbuckets;
  uint32_t* gbase = lstart + ba.nbuckets;
  uint32_t* nin = gbase + ba.nbuckets;
  uint32_t* obase = nin + ba.nbuckets;
  uint32_t* wsum = obase + ba.nbuckets;  // 16 slots
  uint32_t* ltile = wsum + 16;
  const bool lds_tiles = ba.ntiles <= LDS_TILES_MAX;
  if (lds_tiles)
    for (int t = threadIdx.x; t < ba.ntiles; t += NT) ltile[t] = 0u;
  double acc[CNPC_SUMS_LEN];
#pragma unroll
  for (int q = 0; q < CNPC_SUMS_LEN; ++q) acc[q] = 0.0;
  const double scale = sa.boxsize / 4294967296.0;
  const int bshift = 3 * ba.g.ls;
  const int64_t stride = (int64_t)gridDim.x * CH;
  // c < n: indices past the end are clamped to the last particle, so the
  // loads form straight-line code and are all in flight before the first use
  // (a load under a branch is waited for before the next one is issued)
  auto load_chunk = [&](int64_t c, Rec<RS>* dst) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t i = min(c + (int64_t)k * NT + threadIdx.x, n - 1);
      dst[k].v[0] = pos[i];
      dst[k].v[1] = pos[n + i];
      dst[k].v[2] = pos[2 * n + i];
      if constexpr (RS == 4) dst[k].v[3] = __float_as_uint(w[i]);
    }
  };
  uint16_t* stile = reinterpret_cast<uint16_t*>(ltile + (lds_tiles ? ba.ntiles : 0));  // [CH] (pack)
  Rec<RS> rn[PF ? PER : 1];
  if constexpr (PF) load_chunk((int64_t)blockIdx.x * CH, rn);
  for (int64_t c0 = (int64_t)blockIdx.x * CH; c0 < n; c0 += stride) {
    Rec<RS> r[PER];
    int key[PER];
    __syncthreads();  // the previous chunk's LDS reads are done
    for (int t = threadIdx.x; t < ba.nbuckets; t += NT) hist[t] = 0u;
#pragma unroll
    for (int k = 0; k < PER; ++k) key[k] = -1;
    if constexpr (PF) {
#pragma unroll
      for (int k = 0; k < PER; ++k) r[k] = rn[k];
      if (c0 + stride < n) load_chunk(c0 + stride, rn);
    } else {
      load_chunk(c0, r);
    }
    __syncthreads();
    uint32_t rank[PER];
    int tk[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t i = c0 + (int64_t)k * NT + threadIdx.x;
      tk[k] = 0;
      if (i < n) {
        const int t = tile_key(r[k].v[0], r[k].v[1], r[k].v[2], ba.g);
        tk[k] = t;
        key[k] = t >> bshift;
        if (lds_tiles) atomicAdd(&ltile[t], 1u);
        else atomicAdd(&ba.tcount[t], 1u);
        rank[k] = atomicAdd(&hist[key[k]], 1u);
        const double wi = RS == 4 ? (double)__uint_as_float(r[k].v[3]) : 1.0;
        sums_add<LMAX>(acc, r[k].v[0], r[k].v[1], r[k].v[2], wi, scale, sa);
      }
    }
    __syncthreads();
    block_exclusive_scan<NT>(hist, ba.nbuckets, wsum, [&](int b, uint32_t v) {
      lstart[b] = v;
      const uint32_t c = hist[b];
      uint32_t gb = 0u, ni = 0u, ob = 0u;
      if (c) {
        gb = atomicAdd(&ba.bcnt[b], c);
        ni = gb >= ba.cap ? 0u : min(c, ba.cap - gb);
        if (c > ni) ob = atomicAdd(ba.ovf, c - ni);
      }
      gbase[b] = gb;
      nin[b] = ni;
      obase[b] = ob;
    });
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (key[k] >= 0) {
        const uint32_t slot = lstart[key[k]] + rank[k];
        stage[slot] = r[k];
        skey[slot] = (uint16_t)key[k];
        if (ba.pack) stile[slot] = (uint16_t)tk[k];
      }
    __syncthreads();
    const int cnt = (int)min((int64_t)CH, n - c0);
    if (RS == 3 && ba.pack) {
      for (int j = threadIdx.x; j < cnt; j += NT) {
        const int b = skey[j];
        const uint32_t q = (uint32_t)j - lstart[b];
        const uint64_t v = pack_rec(*reinterpret_cast<const Rec<3>*>(&stage[j]), ba.g.shift);
        if (q < nin[b]) {
          const int64_t o = (int64_t)b * ba.cap + gbase[b] + q;
          reinterpret_cast<uint64_t*>(region)[o] = v;
          ba.rkey[o] = stile[j];
        } else {
          const int64_t o = obase[b] + (q - nin[b]);
          reinterpret_cast<uint64_t*>(ovf_out)[o] = v;
          ba.okey[o] = stile[j];
        }
      }
    } else {
      for (int j = threadIdx.x; j < cnt; j += NT) {
        const int b = skey[j];
        const uint32_t q = (uint32_t)j - lstart[b];
        if (q < nin[b]) region[(int64_t)b * ba.cap + gbase[b] + q] = stage[j];
        else ovf_out[obase[b] + (q - nin[b])] = stage[j];
      }
    }
  }
  // catalog-sum partial of the workgroup (fixed-order reduction)
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem_raw);  // [NT / 64][CNPC_SUMS_LEN], over the stage
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CNPC_SUMS_LEN; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) red[wv * CNPC_SUMS_LEN + q] = v;
  }
  __syncthreads();
  if (threadIdx.x < CNPC_SUMS_LEN) {
    double v = 0.0;
    for (int k = 0; k < NT / 64; ++k) v += red[k * CNPC_SUMS_LEN + threadIdx.x];
    ba.partial[(int64_t)blockIdx.x * CNPC_SUMS_LEN + threadIdx.x] = v;
  }
  if (lds_tiles)
    for (int t = threadIdx.x; t < ba.ntiles; t += NT) {
      const uint32_t c = ltile[t];
      if (c) atomicAdd(&ba.tcount[t], c);
    }
}

// Second counting-sort step over the bucket regions: workgroup (b, j) sorts
// records j CH .. of bucket b (its keys lie in bucket b); workgroups past the
// last region chunk walk the overflow records (mixed buckets: one global slot
// per particle).
template <int RS, int PER, int NT>
__global__ void __launch_bounds__(NT) k_tile_pass(const Rec<RS>* __restrict__ region,
                                                  const Rec<RS>* __restrict__ ovf_in, const uint32_t* __restrict__ bcnt,
                                                  const uint32_t* __restrict__ ovf, uint32_t cap, int chunks_per_bucket,
                                                  int nbuckets, TileGeom g, uint32_t* __restrict__ cursor,
                                                  Rec<RS>* __restrict__ rout, bool pack) {
  constexpr int CH = NT * PER;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bshift = 3 * g.ls;
  const int R = 1 << bshift;  // tiles per bucket
  const int nreg = nbuckets * chunks_per_bucket;
  if ((int)blockIdx.x >= nreg) {
    const uint32_t no = *ovf;
    for (int64_t c0 = (int64_t)(blockIdx.x - nreg) * CH; c0 < no; c0 += (int64_t)(gridDim.x - nreg) * CH) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int64_t i = c0 + (int64_t)k * NT + threadIdx.x;
        if (i < no) {
          const Rec<RS> rr = ovf_in[i];
          put_rec(rout, atomicAdd(&cursor[tile_key(rr.v[0], rr.v[1], rr.v[2], g)], 1u), rr, pack, g.shift);
        }
      }
    }
    return;
  }
  const int b = blockIdx.x / chunks_per_bucket, jc = blockIdx.x - b * chunks_per_bucket;
  const uint32_t nb_ = min(bcnt[b], cap);
  const int64_t c0 = (int64_t)jc * CH;
  if (c0 >= nb_) return;
  const int cnt = (int)min((int64_t)CH, (int64_t)nb_ - c0);
  const Rec<RS>* rin = region + (int64_t)b * cap + c0;
  Rec<RS>* stage = reinterpret_cast<Rec<RS>*>(smem_raw);                        // [CH]
  uint16_t* skey = reinterpret_cast<uint16_t*>(smem_raw + (size_t)CH * RS * 4);  // [CH]
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem_raw + (size_t)CH * (RS * 4 + 2));
  uint32_t* lstart = hist + R;
  uint32_t* gbase = lstart + R;
  uint32_t* wsum = gbase + R;  // 16 slots
  const int klo = b << bshift;
  Rec<RS> r[PER];
  int key[PER];
  // cnt >= 1: clamped straight-line loads, all in flight before the first use
#pragma unroll
  for (int k = 0; k < PER; ++k) r[k] = rin[min(k * NT + (int)threadIdx.x, cnt - 1)];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    key[k] = k * NT + (int)threadIdx.x < cnt ? tile_key(r[k].v[0], r[k].v[1], r[k].v[2], g) - klo : -1;
  for (int t = threadIdx.x; t < R; t += NT) hist[t] = 0u;
  __syncthreads();
  uint32_t rank[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) rank[k] = atomicAdd(&hist[key[k]], 1u);
  __syncthreads();
  block_exclusive_scan<NT>(hist, R, wsum, [&](int t, uint32_t v) {
    lstart[t] = v;
    const uint32_t c = hist[t];
    gbase[t] = c ? atomicAdd(&cursor[klo + t], c) : 0u;
  });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) {
      const uint32_t slot = lstart[key[k]] + rank[k];
      stage[slot] = r[k];
      skey[slot] = (uint16_t)key[k];
    }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += NT) {
    const int kk = skey[j];
    put_rec(rout, gbase[kk] + (j - lstart[kk]), stage[j], pack, g.shift);
  }
}

// k_tile_pass over records the bucket pass wrote packed (pack_rec + 16-bit tile
// index, for the FP32 painter): the tile index comes from its own array and the
// packed records are moved as they are
template <int PER, int NT>
__global__ void __launch_bounds__(NT) k_tile_pass_packed(const uint64_t* __restrict__ region,
                                                         const uint16_t* __restrict__ rkey,
                                                         const uint64_t* __restrict__ ovf_in,
                                                         const uint16_t* __restrict__ okey,
                                                         const uint32_t* __restrict__ bcnt,
                                                         const uint32_t* __restrict__ ovf, uint32_t cap,
                                                         int chunks_per_bucket, int nbuckets, TileGeom g,
                                                         uint32_t* __restrict__ cursor, uint64_t* __restrict__ rout) {
  constexpr int CH = NT * PER;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bshift = 3 * g.ls;
  const int R = 1 << bshift;
  const int nreg = nbuckets * chunks_per_bucket;
  if ((int)blockIdx.x >= nreg) {
    const uint32_t no = *ovf;
    for (int64_t c0 = (int64_t)(blockIdx.x - nreg) * CH; c0 < no; c0 += (int64_t)(gridDim.x - nreg) * CH) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int64_t i = c0 + (int64_t)k * NT + threadIdx.x;
        if (i < no) rout[atomicAdd(&cursor[okey[i]], 1u)] = ovf_in[i];
      }
    }
    return;
  }
  const int b = blockIdx.x / chunks_per_bucket, jc = blockIdx.x - b * chunks_per_bucket;
  const uint32_t nb_ = min(bcnt[b], cap);
  const int64_t c0 = (int64_t)jc * CH;
  if (c0 >= nb_) return;
  const int cnt = (int)min((int64_t)CH, (int64_t)nb_ - c0);
  const uint64_t* rin = region + (int64_t)b * cap + c0;
  const uint16_t* kin = rkey + (int64_t)b * cap + c0;
  uint64_t* stage = reinterpret_cast<uint64_t*>(smem_raw);                  // [CH]
  uint16_t* skey = reinterpret_cast<uint16_t*>(smem_raw + (size_t)CH * 8);  // [CH]
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem_raw + (size_t)CH * 10);
  uint32_t* lstart = hist + R;
  uint32_t* gbase = lstart + R;
  uint32_t* wsum = gbase + R;  // 16 slots
  const int klo = b << bshift;
  uint64_t r[PER];
  int key[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ii = min(k * NT + (int)threadIdx.x, cnt - 1);
    r[k] = rin[ii];
    key[k] = (int)kin[ii];
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) key[k] = k * NT + (int)threadIdx.x < cnt ? key[k] - klo : -1;
  for (int t = threadIdx.x; t < R; t += NT) hist[t] = 0u;
  __syncthreads();
  uint32_t rank[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) rank[k] = atomicAdd(&hist[key[k]], 1u);
  __syncthreads();
  block_exclusive_scan<NT>(hist, R, wsum, [&](int t, uint32_t v) {
    lstart[t] = v;
    const uint32_t c = hist[t];
    gbase[t] = c ? atomicAdd(&cursor[klo + t], c) : 0u;
  });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (key[k] >= 0) {
      const uint32_t slot = lstart[key[k]] + rank[k];
      stage[slot] = r[k];
      skey[slot] = (uint16_t)key[k];
    }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += NT) {
    const int kk = skey[j];
    rout[gbase[kk] + (j - lstart[kk])] = stage[j];
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

template <typename T, int ASSIGN, int RS>
__global__ void __launch_bounds__(1024) k_paint_tiles(const Rec<RS>* __restrict__ rec,
                                                     const uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ count, TileGeom g,
                                                     int nphase, int ph0, int nph, int power,
                                                     T* __restrict__ blocks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem_raw);  // [nph][BVOL]
  const int t = blockIdx.x;  // tile (tx * nt + ty) * nt + tz
  const int shift = g.shift;
  for (int i = threadIdx.x; i < nph * BVOL; i += blockDim.x) acc[i] = 0ull;
  __syncthreads();
  const int key = key_of(t / (g.nt * g.nt), (t / g.nt) % g.nt, t % g.nt, g);
  const uint32_t s0 = start[key], cnt = count[key];
  constexpr int NP = ASSIGN == CNPC_TSC ? 3 : 2;
  for (uint32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
    const Rec<RS> p = rec[(int64_t)s0 + k];
    const uint32_t px = p.v[0], py = p.v[1], pz = p.v[2];
    T wv = T(1);
    if constexpr (RS == 4) {
      wv = T(__uint_as_float(p.v[3]));
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
      // node lz = bz + oz + iz sits at lz - 1 in its row, lz = 0 at 18
      const int a1 = q * BVOL + (bx + ox) * BW * BW + (by + oy) * BW + (bz + oz - 1);
      const int a0 = a1 + (bz + oz == 0 ? BW : 0);
#pragma unroll
      for (int ix = 0; ix < NP; ++ix) {
        const T vx = wv * wx[ix];
#pragma unroll
        for (int iy = 0; iy < NP; ++iy) {
          const T vxy = vx * wy[iy];
#pragma unroll
          for (int iz = 0; iz < NP; ++iz) {
            const long long fixv = __double2ll_rn((double)(vxy * wz[iz]) * FIX_SCALE);
            atomicAdd(&acc[(iz == 0 ? a0 : a1) + ix * BW * BW + iy * BW + iz], (unsigned long long)fixv);
          }
        }
      }
    }
  }
  __syncthreads();
  T* out = blocks + ((int64_t)t * nphase + ph0) * BSTRIDE;
  for (int i = threadIdx.x; i < nph * BVOL; i += blockDim.x) {
    const int q = i >= BVOL ? 1 : 0;
    out[q * BSTRIDE + i - q * BVOL] = T((double)(long long)acc[i] * FIX_INV);
  }
}

// Unit-weight FP32 painting with 32-bit LDS atomics.  Each round of the
// workgroup paints one particle per thread; a node then gains at most
// PPF * max node weight per flush interval (PPF = particles per flush), which
// at 2^21 units stays below 2^32 (TSC: 4096 * 0.421875 * 2^21; CIC:
// 1024 * 1 * 2^21), so the 32-bit sums are exact.  After every interval each
// thread moves the nodes it owns into 64-bit registers and clears them.  The
// result equals the 64-bit fixed-point sum of the contributions rounded to
// 2^-21 (half up), independent of the order of the additions.  From 256^3 up
// the particles come as packed 8-byte records (pack_rec): positions inside the
// tile on a 2^-17 cell grid.
constexpr int PAINT32_THREADS = 1024;
constexpr int PAINT32_OWN = (2 * BVOL + PAINT32_THREADS - 1) / PAINT32_THREADS;  // nodes per thread

// 1-D stencil in 32-bit integer arithmetic (shift <= 28): same nodes and
// weights as stencil_1d<float>, times `scale`, a power of two (scaling by it
// is exact, so a scaled weight is bit for bit the scaled unscaled weight).
template <int ASSIGN>
__device__ __forceinline__ int stencil32(uint32_t p, int shift, int phase, float* wt, float scale = 1.0f) {
  const uint32_t one = 1u << shift, half = one >> 1;
  const int f = (int)(p & (one - 1u));
  const float inv = 1.0f / (float)one;
  if constexpr (ASSIGN == CNPC_TSC) {
    int off, dfix;
    if (phase == 0) {
      const bool up = f >= (int)half;
      off = up ? 1 : 0;
      dfix = up ? f - (int)one : f;
    } else {
      off = 0;
      dfix = f - (int)half;
    }
    const float d = (float)dfix * inv;
    const float a = 0.5f - d, b = 0.5f + d;
    wt[0] = (0.5f * scale) * a * a;
    wt[1] = __builtin_fmaf(-d, d * scale, 0.75f * scale);
    wt[2] = (0.5f * scale) * b * b;
    return off - 1;
  } else {
    if (phase == 0) {
      const float d = (float)f * inv;
      wt[0] = __builtin_fmaf(-d, scale, scale);
      wt[1] = d * scale;
      return 0;
    }
    const bool up = f >= (int)half;
    const int off = up ? 0 : -1;
    const int dfix = up ? f - (int)half : f + (int)half;
    const float d = (float)dfix * inv;
    wt[0] = __builtin_fmaf(-d, scale, scale);
    wt[1] = d * scale;
    return off;
  }
}

template <int ASSIGN>
__global__ void __launch_bounds__(PAINT32_THREADS, 8) k_paint_tiles_u32(const Rec<3>* __restrict__ rec,
                                                                     const uint32_t* __restrict__ start,
                                                                     const uint32_t* __restrict__ count,
                                                                     TileGeom g, int nphase, bool packed,
                                                                     float* __restrict__ blocks) {
  constexpr float SCALE = 2097152.0f;  // 2^21
  constexpr int ROUNDS_PER_FLUSH = ASSIGN == CNPC_TSC ? 4 : 1;
  constexpr int NP = ASSIGN == CNPC_TSC ? 3 : 2;
  __shared__ __align__(16) uint32_t acc[2 * BVOL];
  const int t = blockIdx.x;
  const int shift = g.shift;
  const int nv = nphase * BVOL;
  for (int i = threadIdx.x; i < nv; i += PAINT32_THREADS) acc[i] = 0u;
  unsigned long long own[PAINT32_OWN];
#pragma unroll
  for (int j = 0; j < PAINT32_OWN; ++j) own[j] = 0ull;
  __syncthreads();
  const int key = key_of(t / (g.nt * g.nt), (t / g.nt) % g.nt, t % g.nt, g);
  const uint32_t s0 = start[key], cnt = count[key];
  int round = 0;
  for (uint32_t base = 0; base < cnt; base += PAINT32_THREADS) {
    const uint32_t k = base + threadIdx.x;
    if (k < cnt) {
      uint32_t px, py, pz;
      if (packed) {  // pack_rec: tile-relative positions on the 2^-17 cell grid
        const uint64_t q = reinterpret_cast<const uint64_t*>(rec)[(int64_t)s0 + k];
        const int up = shift - 17;
        px = (uint32_t)(q & 0x1fffffu) << up;
        py = (uint32_t)((q >> 21) & 0x1fffffu) << up;
        pz = (uint32_t)((q >> 42) & 0x1fffffu) << up;
      } else {
        const Rec<3> p = rec[(int64_t)s0 + k];
        px = p.v[0];
        py = p.v[1];
        pz = p.v[2];
      }
      const int bx = ((int)(px >> shift) & 15) + 1;
      const int by = ((int)(py >> shift) & 15) + 1;
      const int bz = ((int)(pz >> shift) & 15) + 1;
      for (int ph = 0; ph < nphase; ++ph) {
        float wx[3], wy[3], wz[3];
        const int ox = stencil32<ASSIGN>(px, shift, ph, wx, SCALE);  // x weights carry the 2^21 units
        const int oy = stencil32<ASSIGN>(py, shift, ph, wy);
        const int oz = stencil32<ASSIGN>(pz, shift, ph, wz);
        // node lz = bz + oz + iz sits at lz - 1 in its row, lz = 0 at 18
        const int a1 = ph * BVOL + (bx + ox) * BW * BW + (by + oy) * BW + (bz + oz - 1);
        const int a0 = a1 + (bz + oz == 0 ? BW : 0);
#pragma unroll
        for (int ix = 0; ix < NP; ++ix)
#pragma unroll
          for (int iy = 0; iy < NP; ++iy) {
            const float vxy = wx[ix] * wy[iy];
            const int o = ix * BW * BW + iy * BW;
#pragma unroll
            for (int iz = 0; iz < NP; ++iz)
              atomicAdd(&acc[(iz == 0 ? a0 : a1) + o + iz], (uint32_t)__builtin_fmaf(vxy, wz[iz], 0.5f));
          }
      }
    }
    if (++round == ROUNDS_PER_FLUSH || base + PAINT32_THREADS >= cnt) {
      round = 0;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < PAINT32_OWN; ++j) {
        const int i = threadIdx.x + j * PAINT32_THREADS;
        if (i < nv) {
          own[j] += acc[i];
          acc[i] = 0u;
        }
      }
      __syncthreads();
    }
  }
  float* out = blocks + (int64_t)t * nphase * BSTRIDE;
#pragma unroll
  for (int j = 0; j < PAINT32_OWN; ++j) {
    const int i = threadIdx.x + j * PAINT32_THREADS;
    if (i < nv) {
      const int q = i >= BVOL ? 1 : 0;
      out[q * BSTRIDE + i - q * BVOL] = (float)((double)own[j] * (1.0 / (double)SCALE));
    }
  }
}

// 16 consecutive elements from an address aligned to the element size
// (gfx950 takes 16-byte loads at 4-byte alignment)
template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ p, T* v) {
  struct __attribute__((aligned(sizeof(T)))) V2 { T a, b; };
  struct __attribute__((aligned(sizeof(T)))) V4 { T a, b, c, d; };
  if constexpr (sizeof(T) == 4) {
    const V4* q = reinterpret_cast<const V4*>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const V4 u = q[k];
      v[4 * k] = u.a; v[4 * k + 1] = u.b; v[4 * k + 2] = u.c; v[4 * k + 3] = u.d;
    }
  } else {
    const V2* q = reinterpret_cast<const V2*>(p);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const V2 u = q[k];
      v[2 * k] = u.a; v[2 * k + 1] = u.b;
    }
  }
}

// 16 consecutive elements to a 16 * sizeof(T)-aligned address
template <typename T>
__device__ __forceinline__ void store16(T* __restrict__ p, const T* v) {
  if constexpr (sizeof(T) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  } else {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = make_double2(v[2 * k], v[2 * k + 1]);
  }
}

// Fold of the tile blocks into meshes.  A workgroup covers Z2 tiles along z
// of one (x, y) tile column and one phase; a thread owns the 16-node z-row
// (x, y) of one tile.  Along x (and y) the row gathers from its own tile
// (local row l = c + 1) and, for c = 0, 1 (15), from the lower neighbour's
// row l = c + 17 (the upper neighbour's row 0); from each of these <= 4 (x, y)
// sources it reads the 16 own values of the row in the same z tile, values
// 16..17 of the row in the lower z tile (nodes 0, 1) and value 18 of the row
// in the upper z tile (node 15): every block element is read exactly once.
// Per set the sum is formed first, then delta = sum_s cd[s] v_s and
// N = sum_s cn[s] v_s.
template <typename T>
__global__ void __launch_bounds__(512) k_fold_tiles(FoldArgs<T> fa, const double* __restrict__ norms,
                                                    T* __restrict__ delta, T* __restrict__ noise) {
  const int n = fa.n, nt = fa.nt, z2 = nt >= 2 ? 2 : 1;
  const int nzp = nt / z2;
  // workgroups go to the 8 XCDs in turn (launch index mod 8); give each XCD a
  // contiguous range of tile columns so that the halo rows shared by
  // neighbouring tiles are fetched into one L2 (a bijection when 8 | grid)
  int b = blockIdx.x;
  if ((gridDim.x & 7u) == 0) b = (int)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  const int tzp = b % nzp; b /= nzp;
  const int ty = b % nt; b /= nt;
  const int tx = b % nt;
  const int ph = b / nt;
  const int zt = threadIdx.x % z2, row = threadIdx.x / z2;
  const int cx = row >> 4, cy = row & 15;
  const int tz = tzp * z2 + zt;
  const double alpha = norms[CNPC_NORM_ALPHA];
  T cd[4] = {T(0), T(0), T(0), T(0)}, cn[4] = {T(0), T(0), T(0), T(0)};
  if (fa.nsets == 2) {
    cd[0] = T(1); cd[1] = T(-alpha); cn[0] = T(1); cn[1] = T(alpha * alpha);
  } else {
    cd[0] = T(1); cd[1] = T(-alpha); cn[2] = T(1); cn[3] = T(alpha * alpha);
  }
  // x / y sources: own tile (row c + 1) or, near the faces, the neighbour
  const bool hx = cx <= 1 || cx == 15, hy = cy <= 1 || cy == 15;
  const int txn = cx <= 1 ? (tx - 1 + nt) % nt : (tx + 1) % nt;
  const int tyn = cy <= 1 ? (ty - 1 + nt) % nt : (ty + 1) % nt;
  const int lxn = cx <= 1 ? cx + 17 : 0, lyn = cy <= 1 ? cy + 17 : 0;
  const int tzl = (tz - 1 + nt) % nt, tzu = (tz + 1) % nt;
  const int64_t bst = (int64_t)fa.nphase * BSTRIDE;  // per tile
  // element offsets of the row of source k = 2 a + c (a: x neighbour, c: y
  // neighbour) in the same, lower and upper z tile; source k is used when ok[k]
  int64_t o0[4], o1[4], o2[4];
  bool ok[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int a = k >> 1, c = k & 1;
    ok[k] = (!a || hx) && (!c || hy);
    const int txs = a ? txn : tx, tys = c ? tyn : ty;
    const int r = ((a ? lxn : cx + 1) * BW + (c ? lyn : cy + 1)) * BW;
    const int64_t col = ((int64_t)txs * nt + tys) * nt;
    o0[k] = (col + tz) * bst + (int64_t)ph * BSTRIDE + r;
    o1[k] = (col + tzl) * bst + (int64_t)ph * BSTRIDE + r + 16;
    o2[k] = (col + tzu) * bst + (int64_t)ph * BSTRIDE + r + 18;
  }
  T d[16], q[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) d[e] = q[e] = T(0);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s >= fa.nsets) break;
    const T* __restrict__ bl = fa.blocks[s];
    T v[16];
    load16<T>(bl + o0[0], v);
    T lo0 = bl[o1[0]], lo1 = bl[o1[0] + 1], up = bl[o2[0]];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      if (!ok[k]) continue;
      T u[16];
      load16<T>(bl + o0[k], u);
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] += u[e];
      lo0 += bl[o1[k]];
      lo1 += bl[o1[k] + 1];
      up += bl[o2[k]];
    }
    v[0] += lo0;
    v[1] += lo1;
    v[15] += up;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      d[e] += cd[s] * v[e];
      q[e] += cn[s] * v[e];
    }
  }
  const int64_t idx = (int64_t)ph * n * n * n + ((int64_t)(tx * 16 + cx) * n + ty * 16 + cy) * n + tz * 16;
  store16<T>(delta + idx, d);
  if (noise) store16<T>(noise + idx, q);
}

// Fold fused with the z pass of the de-interlacing transforms (N = 256: 16
// z-tiles, one z-row = one row_fft_rr of 16 lanes).  A workgroup takes the 16
// node rows (x, y = 16 ty + cy) of one x node x = 16 tx + cx of the tile
// column (ph, tx, ty).  Load phase, lane (cy, tz): the block rows that hold
// the 16 nodes of z-tile tz of row cy (own tile, the x / y neighbours' halo
// rows; rows of consecutive cy are contiguous in a block, so 16 lanes read
// 16 x 19 consecutive elements) are summed over the sources, and over both
// weight sets into delta = sum cd v and N = sum cn v, then staged in LDS; the
// row's z halo (positions 16, 17: nodes 0, 1 of z-tile tz + 1; position 18:
// node 15 of z-tile tz - 1) is added after a barrier, one writer per node.
// Transform phase: group g transforms row g (delta + i N) and the two-for-one
// split gives the r2c z transforms of delta (kz < kz_d) and N (kz < kz_n).
// Sources that a lane does not need are read from its own row and weighted by
// zero, so no load sits in a divergent branch.  The meshes are never written.
constexpr int FZ_RS = 273;  // staged row stride (complex): 256 nodes + 1 pad per 16

template <typename T>
__global__ void __launch_bounds__(256) k_fold_zr2c(FoldArgs<T> fa, const double* __restrict__ norms,
                                                   cx<T>* __restrict__ dsp, int kz_d, cx<T>* __restrict__ nw1,
                                                   int kz_n) {
  constexpr int R = 16, N = 256;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* stage = tw + N;  // [16][FZ_RS]; later the row_fft_rr buffers
  load_twiddles<T, N, -1>(tw);
  // workgroups go to the 8 XCDs in turn: each XCD takes a contiguous range of
  // tile columns, so the blocks and halo rows they share meet in one L2
  int b = blockIdx.x;
  if ((gridDim.x & 7u) == 0) b = (int)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  const int nt = fa.nt;
  const int cx_ = b & 15;
  b >>= 4;
  const int ty = b % nt;
  b /= nt;
  const int tx = b % nt;
  const int ph = b / nt;
  const int tz = threadIdx.x >> 4, cy = threadIdx.x & 15;
  const double alpha = norms[CNPC_NORM_ALPHA];
  T cd[4] = {T(0), T(0), T(0), T(0)}, cn[4] = {T(0), T(0), T(0), T(0)};
  if (fa.nsets == 2) {
    cd[0] = T(1); cd[1] = T(-alpha); cn[0] = T(1); cn[1] = T(alpha * alpha);
  } else {
    cd[0] = T(1); cd[1] = T(-alpha); cn[2] = T(1); cn[3] = T(alpha * alpha);
  }
  // hx is uniform over the workgroup; a lane without a y halo reads its own
  // row for the y-neighbour sources and weighs them by fy = 0
  const bool hx = cx_ <= 1 || cx_ == 15, hy = cy <= 1 || cy == 15;
  const int txn = cx_ <= 1 ? (tx - 1 + nt) % nt : (tx + 1) % nt;
  const int tyn = cy <= 1 ? (ty - 1 + nt) % nt : (ty + 1) % nt;
  const int lxn = cx_ <= 1 ? cx_ + 17 : 0, lyn = cy <= 1 ? cy + 17 : 0;
  const int64_t bst = (int64_t)fa.nphase * BSTRIDE;
  int64_t o[4];  // source k = 2 a + c (a: x neighbour, c: y neighbour)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int a = k >> 1;
    const bool c = (k & 1) && hy;
    const int txs = a ? txn : tx, tys = c ? tyn : ty;
    const int r = ((a ? lxn : cx_ + 1) * BW + (c ? lyn : cy + 1)) * BW;
    o[k] = (((int64_t)txs * nt + tys) * nt + tz) * bst + (int64_t)ph * BSTRIDE + r;
  }
  const T fy = hy ? T(1) : T(0);
  T d[19], q[19];
#pragma unroll
  for (int e = 0; e < 19; ++e) d[e] = q[e] = T(0);
#pragma unroll
  for (int sidx = 0; sidx < 4; ++sidx) {
    if (sidx >= fa.nsets) break;
    const T* __restrict__ bl = fa.blocks[sidx];
    T v[19], u[19];
    load16<T>(bl + o[0], v);
    v[16] = bl[o[0] + 16]; v[17] = bl[o[0] + 17]; v[18] = bl[o[0] + 18];
    load16<T>(bl + o[1], u);
    u[16] = bl[o[1] + 16]; u[17] = bl[o[1] + 17]; u[18] = bl[o[1] + 18];
#pragma unroll
    for (int e = 0; e < 19; ++e) v[e] += fy * u[e];
    if (hx) {
      load16<T>(bl + o[2], u);
      u[16] = bl[o[2] + 16]; u[17] = bl[o[2] + 17]; u[18] = bl[o[2] + 18];
#pragma unroll
      for (int e = 0; e < 19; ++e) v[e] += u[e];
      load16<T>(bl + o[3], u);
      u[16] = bl[o[3] + 16]; u[17] = bl[o[3] + 17]; u[18] = bl[o[3] + 18];
#pragma unroll
      for (int e = 0; e < 19; ++e) v[e] += fy * u[e];
    }
#pragma unroll
    for (int e = 0; e < 19; ++e) {
      d[e] += cd[sidx] * v[e];
      q[e] += cn[sidx] * v[e];
    }
  }
  // staged node (row, z) at row * FZ_RS + z + z / 16
  cx<T>* srow = stage + cy * FZ_RS;
#pragma unroll
  for (int e = 0; e < 16; ++e) srow[17 * tz + e] = cx<T>{d[e], q[e]};
  __syncthreads();
  {
    cx<T>* up = srow + 17 * ((tz + 1) & 15);
    cx<T>* lo = srow + 17 * ((tz + 15) & 15) + 15;
    up[0] = cadd(up[0], cx<T>{d[16], q[16]});
    up[1] = cadd(up[1], cx<T>{d[17], q[17]});
    *lo = cadd(*lo, cx<T>{d[18], q[18]});
  }
  __syncthreads();
  const int grp = threadIdx.x >> 4, rank = threadIdx.x & 15;
  cx<T> v[R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) v[n2] = stage[grp * FZ_RS + 17 * n2 + rank];
  __syncthreads();
  row_fft_rr<T, R, -1>(v, rank, stage + grp * (R * (R + 1)), tw);
  const int src = (R - rank) & (R - 1);
  const int kzmax = kz_d > kz_n ? kz_d : kz_n;
  const int K2 = (kzmax + R - 1) / R;
  const int64_t row = ((int64_t)ph * N + 16 * tx + cx_) * N + 16 * ty + grp;
  cx<T>* od = dsp + row * kz_d;
  cx<T>* on = nw1 + row * kz_n;
#pragma unroll
  for (int k2 = 0; k2 < R / 2; ++k2) {
    if (k2 < K2) {
      const cx<T> a = v[R - 1 - k2];
      const cx<T> sh = {__shfl(a.x, src, R), __shfl(a.y, src, R)};
      const cx<T> zm = cconj(rank ? sh : v[(R - k2) & (R - 1)]);
      const cx<T> zk = v[k2];
      const int k = rank + R * k2;
      const cx<T> dd = csub(zk, zm);
      if (k < kz_d) od[k] = cscale(cadd(zk, zm), T(0.5));
      if (k < kz_n) on[k] = cx<T>{T(0.5) * dd.y, T(-0.5) * dd.x};
    }
  }
}

// ------------------------------------------------------------------- host --
static TileGeom tile_geom(const cnpc_mesh_desc* d);

static cnpc_status sums_counted(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w, int64_t n,
                                int lmax, double* sums, double* partial, const CountArgs& ca, hipStream_t s) {
  const int nblocks = SUMS_BLOCKS;
  SumsArgs a;
  a.lmax = lmax;
  a.boxsize = d->boxsize;
  for (int i = 0; i < 3; ++i) { a.obs[i] = d->observer[i]; a.los[i] = d->los[i]; }
  a.global_los = d->los_mode == CNPC_LOS_GLOBAL;
  const size_t lds = (ca.count && ca.ntiles <= LDS_TILES_MAX) ? (size_t)ca.ntiles * 4 : 0;
  kt_begin(CNPC_KT_SUMS, s);
  if (lmax >= 4)
    hipLaunchKernelGGL(k_catalog_sums<4>, dim3(nblocks), dim3(SUMS_THREADS), lds, s, pos, w, n, a, partial, ca);
  else if (lmax >= 2)
    hipLaunchKernelGGL(k_catalog_sums<2>, dim3(nblocks), dim3(SUMS_THREADS), lds, s, pos, w, n, a, partial, ca);
  else
    hipLaunchKernelGGL(k_catalog_sums<0>, dim3(nblocks), dim3(SUMS_THREADS), lds, s, pos, w, n, a, partial, ca);
  kt_end(CNPC_KT_SUMS, s);
  CNPC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_partials, dim3(CNPC_SUMS_LEN), dim3(64), 0, s, partial, nblocks, sums);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_catalog_sums(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w,
                                int64_t n, double* sums, void* ws, size_t ws_bytes,
                                hipStream_t s) {
  const int nblocks = SUMS_BLOCKS;
  if (ws_bytes < (size_t)nblocks * CNPC_SUMS_LEN * sizeof(double)) {
    set_error("catalog_sums workspace too small");
    return CNPC_EWORKSPACE;
  }
  CountArgs ca;
  ca.ntiles = 0;
  ca.count = nullptr;
  return sums_counted(d, pos, w, n, 4, sums, reinterpret_cast<double*>(ws), ca, s);
}

cnpc_status launch_norms(const cnpc_mesh_desc* d, const double* gs, const double* rs, int64_t ngal,
                         double* norms, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(64), 0, s, gs, rs, ngal, d->boxsize, norms);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static TileGeom tile_geom(const cnpc_mesh_desc* d) {
  TileGeom g;
  g.shift = 32 - ilog2_host(d->n);
  g.nt = d->n / TILE;
  const int S = g.nt < 4 ? g.nt : 4;
  g.ls = ilog2_host(S);
  g.lnb = ilog2_host(g.nt / S);
  return g;
}

// Bucket-pass geometry: chunk of BUCKET_NT * per particles (per <= 8), at most
// BUCKET_BLOCKS_MAX persistent workgroups; a bucket region holds 1.5 times the
// mean bucket count plus the largest chunk (more goes to the overflow region).
constexpr int BUCKET_NT = 1024;
constexpr int BUCKET_BLOCKS_MAX = 512;
constexpr int OVF_BLOCKS = 256;  // tile-pass workgroups walking the overflow records
static uint32_t bucket_cap(int64_t n, int nbuckets) {
  const int64_t mean = (n + nbuckets - 1) / nbuckets;
  const int64_t c = mean + mean / 2 + (int64_t)BUCKET_NT * 8;
  return (uint32_t)((c + 63) / 64 * 64);
}

PaintLayout paint_layout(const cnpc_mesh_desc* d, int64_t ngal, int64_t nran, bool weighted) {
  PaintLayout L;
  const int nt = d->n / TILE;
  L.nt = nt;
  L.ntiles = nt * nt * nt;
  L.nphase = d->interlace ? 2 : 1;
  L.nsets = weighted ? 4 : 2;
  const TileGeom g = tile_geom(d);
  L.nbuckets = 1 << (3 * g.lnb);
  const size_t es = esize(d->dtype);
  const int64_t np = ngal > nran ? ngal : nran;
  const size_t rec = (size_t)np * (weighted ? 16 : 12);
  size_t off = 0;
  L.off_rec = off; off = align_up(off + rec);
  L.off_tmp = off; off = align_up(off + (L.nbuckets > 1 ? rec : 0));
  L.off_count[0] = off; off = align_up(off + (size_t)L.ntiles * 4);
  L.off_count[1] = off; off = align_up(off + (size_t)L.ntiles * 4);
  L.off_partial = off; off = align_up(off + (size_t)BUCKET_BLOCKS_MAX * CNPC_SUMS_LEN * 8);
  L.off_sums = off; off = align_up(off + (size_t)2 * CNPC_SUMS_LEN * 8);
  L.off_start = off; off = align_up(off + (size_t)L.ntiles * 4);
  L.off_cursor = off; off = align_up(off + (size_t)L.ntiles * 4);
  L.off_bcur = off; off = align_up(off + (size_t)L.nbuckets * 4);
  for (int k = 0; k < L.nsets; ++k) {
    L.off_blocks[k] = off;
    off = align_up(off + (size_t)L.ntiles * L.nphase * BSTRIDE * es);
  }
  L.cap = 0;
  L.off_region = L.off_ovf = L.off_bcnt = off;
  if (L.nbuckets > 1) {
    const size_t rs = weighted ? 16 : 12;
    L.cap = bucket_cap(np, L.nbuckets);
    L.off_region = off; off = align_up(off + (size_t)L.nbuckets * L.cap * rs);
    L.off_ovf = off; off = align_up(off + (size_t)np * rs);
    L.off_bcnt = off; off = align_up(off + (size_t)(L.nbuckets + 1) * 4);
  }
  L.total = off;
  return L;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

constexpr int FINE_RCAP = 512;  // LDS key range of the second sort step

// Particles per thread for nt-thread workgroups: the tuned value when its LDS
// layout fits, else the largest (4, 2, 1) whose layout lets 32 waves' worth
// of workgroups share a CU, else the largest that fits one.
static int partition_per(int rs, int rcap, int nt) {
  const size_t lim = lds_limit();
  const int tp = tune_value(CNPC_TUNE_SORT_PER);
  if (tp > 0 && partition_lds(tp, rs, rcap, nt) <= lim) return tp;
  const size_t wgs = (size_t)(2048 / nt);
  for (int per = 4; per >= 1; per >>= 1)
    if (wgs * partition_lds(per, rs, rcap, nt) <= lim) return per;
  for (int per = 4; per >= 1; per >>= 1)
    if (partition_lds(per, rs, rcap, nt) <= lim) return per;
  return 0;
}

template <bool SOA, bool FINE, int RS, int NT>
static void launch_partition_nt(int per, unsigned nblk, size_t lds, const uint32_t* pos, const float* w,
                                const Rec<RS>* rin, int64_t n, const TileGeom& g, int rcap, uint32_t* cursor,
                                Rec<RS>* rout, bool pack, hipStream_t s) {
  if (per == 4)
    hipLaunchKernelGGL((k_partition<SOA, FINE, RS, 4, NT>), dim3(nblk), dim3(NT), lds, s, pos, w, rin, n, g,
                       rcap, cursor, rout, pack);
  else if (per == 2)
    hipLaunchKernelGGL((k_partition<SOA, FINE, RS, 2, NT>), dim3(nblk), dim3(NT), lds, s, pos, w, rin, n, g,
                       rcap, cursor, rout, pack);
  else
    hipLaunchKernelGGL((k_partition<SOA, FINE, RS, 1, NT>), dim3(nblk), dim3(NT), lds, s, pos, w, rin, n, g,
                       rcap, cursor, rout, pack);
}

template <bool SOA, bool FINE, int RS>
static cnpc_status launch_partition(const uint32_t* pos, const float* w, const Rec<RS>* rin, int64_t n,
                                    const TileGeom& g, int rcap, uint32_t* cursor, Rec<RS>* rout, bool pack,
                                    hipStream_t s) {
  const int nt = tune_value(CNPC_TUNE_SORT_THREADS) == 512 ? 512 : 1024;
  const int per = partition_per(RS, rcap, nt);
  if (per == 0) {
    set_error("sort: %d keys do not fit the LDS of a workgroup", rcap);
    return CNPC_EINVAL;
  }
  const int64_t ch = (int64_t)nt * per;
  const unsigned nblk = (unsigned)((n + ch - 1) / ch);
  const size_t lds = partition_lds(per, RS, rcap, nt);
  kt_begin(CNPC_KT_SORT, s);
  if (nt == 512)
    launch_partition_nt<SOA, FINE, RS, 512>(per, nblk, lds, pos, w, rin, n, g, rcap, cursor, rout, pack, s);
  else
    launch_partition_nt<SOA, FINE, RS, 1024>(per, nblk, lds, pos, w, rin, n, g, rcap, cursor, rout, pack, s);
  kt_end(CNPC_KT_SORT, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

// Tile painting of tile-sorted records (rec, start, count of set set0).
template <typename T, int RS>
static cnpc_status paint_sorted(const cnpc_mesh_desc* d, bool weighted, int set0, unsigned char* ws,
                                const PaintLayout& L, hipStream_t s) {
  const TileGeom g = tile_geom(d);
  uint32_t* count = reinterpret_cast<uint32_t*>(ws + L.off_count[set0]);
  uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.off_start);
  Rec<RS>* rec = reinterpret_cast<Rec<RS>*>(ws + L.off_rec);
  // phases per launch so that the 64-bit LDS blocks fit the workgroup limit
  const int nph = ((size_t)L.nphase * BVOL * 8 <= lds_limit()) ? L.nphase : 1;
  const size_t lds_paint = (size_t)nph * BVOL * 8;
  const int npow = weighted ? 2 : 1;
  for (int pw = 0; pw < npow; ++pw) {
    T* blocks = reinterpret_cast<T*>(ws + L.off_blocks[set0 + 2 * pw]);
    if constexpr (sizeof(T) == 4 && RS == 3) {
      kt_begin(CNPC_KT_PAINT, s);
      if (d->assign == CNPC_TSC)
        hipLaunchKernelGGL((k_paint_tiles_u32<CNPC_TSC>), dim3(L.ntiles), dim3(PAINT32_THREADS), 0, s, rec, start,
                           count, g, L.nphase, packs_records(true, 3, g.shift), reinterpret_cast<float*>(blocks));
      else
        hipLaunchKernelGGL((k_paint_tiles_u32<CNPC_CIC>), dim3(L.ntiles), dim3(PAINT32_THREADS), 0, s, rec, start,
                           count, g, L.nphase, packs_records(true, 3, g.shift), reinterpret_cast<float*>(blocks));
      kt_end(CNPC_KT_PAINT, s);
      CNPC_HIP(hipGetLastError());
      continue;
    }
    for (int ph0 = 0; ph0 < L.nphase; ph0 += nph) {
      kt_begin(CNPC_KT_PAINT, s);
      if (d->assign == CNPC_TSC)
        hipLaunchKernelGGL((k_paint_tiles<T, CNPC_TSC, RS>), dim3(L.ntiles), dim3(1024), lds_paint, s, rec, start,
                           count, g, L.nphase, ph0, nph, pw + 1, blocks);
      else
        hipLaunchKernelGGL((k_paint_tiles<T, CNPC_CIC, RS>), dim3(L.ntiles), dim3(1024), lds_paint, s, rec, start,
                           count, g, L.nphase, ph0, nph, pw + 1, blocks);
      kt_end(CNPC_KT_PAINT, s);
      CNPC_HIP(hipGetLastError());
    }
  }
  return CNPC_OK;
}

template <typename T, int RS>
static cnpc_status sort_and_paint(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w, int64_t n,
                                  int set0, bool weighted, bool counted, unsigned char* ws,
                                  const PaintLayout& L, hipStream_t s) {
  const TileGeom g = tile_geom(d);
  uint32_t* count = reinterpret_cast<uint32_t*>(ws + L.off_count[set0]);
  uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.off_start);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(ws + L.off_cursor);
  uint32_t* bcur = reinterpret_cast<uint32_t*>(ws + L.off_bcur);
  Rec<RS>* rec = reinterpret_cast<Rec<RS>*>(ws + L.off_rec);
  Rec<RS>* tmp = reinterpret_cast<Rec<RS>*>(ws + L.off_tmp);
  if (!counted) {
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count, (int64_t)L.ntiles);
    CNPC_HIP(hipGetLastError());
    const size_t lds_count = L.ntiles <= LDS_TILES_MAX ? (size_t)L.ntiles * 4 : 0;
    const int64_t chunk = (int64_t)SORT_BLOCK * SORT_PER_THREAD;
    const int64_t nblk = (n + chunk - 1) / chunk;
    kt_begin(CNPC_KT_SORT, s);
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)nblk), dim3(SORT_BLOCK), lds_count, s, pos, n, g, L.ntiles,
                       count);
    kt_end(CNPC_KT_SORT, s);
    CNPC_HIP(hipGetLastError());
  }
  const int per_bucket = 1 << (3 * g.ls);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, count, L.ntiles, per_bucket, start, cursor, bcur);
  CNPC_HIP(hipGetLastError());
  const bool pack = packs_records(sizeof(T) == 4, RS, g.shift);  // records of the FP32 painter
  if (L.nbuckets > 1) {
    CNPC_TRY((launch_partition<true, false, RS>(pos, w, nullptr, n, g, L.nbuckets, bcur, tmp, false, s)));
    CNPC_TRY((launch_partition<false, true, RS>(nullptr, nullptr, tmp, n, g, FINE_RCAP, cursor, rec, pack, s)));
  } else {
    CNPC_TRY((launch_partition<true, true, RS>(pos, w, nullptr, n, g, L.ntiles, cursor, rec, pack, s)));
  }
  return paint_sorted<T, RS>(d, weighted, set0, ws, L, s);
}

// Catalog sums, tile histogram and both sort steps from one read of the
// catalog (fused bucket pass), then the tile painting.  sums: CNPC_SUMS_LEN
// doubles (device).
// Bucket-pass shape: CNPC_TUNE_BUCKET 0 (default) 1024 threads; unweighted
// catalogs with the l = 0 sums 8 particles per thread on at most 256
// workgroups (one per CU: 130 KB of LDS), with Y_lm sums 4 on at most 512;
// weighted catalogs 2 on at most 512.  1: 1024 threads, 2 particles, next
// chunk prefetched; 2: 512 threads, 4 particles, prefetched; 3: 1024 threads,
// 4 particles on at most 512 workgroups.  The prefetching forms exist for
// unweighted catalogs with l = 0 or l <= 4 sums; the rest take 0.
struct BucketShape {
  int nt, per;
  bool pf;
  int maxblk;  // persistent workgroups at most
};
static BucketShape bucket_shape(int rs, int lmax) {
  const int v = tune_value(CNPC_TUNE_BUCKET);
  if (rs == 3 && (lmax == 0 || lmax >= 4)) {
    if (v == 1) return {1024, 2, true, BUCKET_BLOCKS_MAX};
    if (v == 2) return {512, 4, true, BUCKET_BLOCKS_MAX};
  }
  if (rs == 4) return {BUCKET_NT, 2, false, BUCKET_BLOCKS_MAX};
  if (v == 3 || lmax > 0) return {BUCKET_NT, 4, false, BUCKET_BLOCKS_MAX};
  return {BUCKET_NT, 8, false, BUCKET_BLOCKS_MAX / 2};
}

template <int RS, int LMAX>
static void launch_bucket_pass(const BucketShape& b, unsigned nblk, size_t lds, const uint32_t* pos, const float* w,
                               int64_t n, const SumsArgs& sa, const BucketArgs& ba, Rec<RS>* region,
                               Rec<RS>* ovf_out, hipStream_t s) {
  if constexpr (RS == 3) {
    if constexpr (LMAX != 2) {
      if (b.pf && b.nt == 1024) {
        hipLaunchKernelGGL((k_bucket_pass<3, 2, 1024, LMAX, true>), dim3(nblk), dim3(1024), lds, s, pos, w, n, sa,
                           ba, region, ovf_out);
        return;
      }
      if (b.pf) {
        hipLaunchKernelGGL((k_bucket_pass<3, 4, 512, LMAX, true>), dim3(nblk), dim3(512), lds, s, pos, w, n, sa, ba,
                           region, ovf_out);
        return;
      }
    }
    if constexpr (LMAX == 0) {
      if (b.per == 8) {
        hipLaunchKernelGGL((k_bucket_pass<3, 8, BUCKET_NT, 0, false>), dim3(nblk), dim3(BUCKET_NT), lds, s, pos, w,
                           n, sa, ba, region, ovf_out);
        return;
      }
    }
    hipLaunchKernelGGL((k_bucket_pass<3, 4, BUCKET_NT, LMAX, false>), dim3(nblk), dim3(BUCKET_NT), lds, s, pos, w, n,
                       sa, ba, region, ovf_out);
  } else {
    hipLaunchKernelGGL((k_bucket_pass<4, 2, BUCKET_NT, LMAX, false>), dim3(nblk), dim3(BUCKET_NT), lds, s, pos, w, n,
                       sa, ba, region, ovf_out);
  }
}

template <typename T, int RS>
static cnpc_status fused_sort_and_paint(const cnpc_mesh_desc* d, const uint32_t* pos, const float* w, int64_t n,
                                        int set0, bool weighted, int sums_lmax, double* sums, unsigned char* ws,
                                        const PaintLayout& L, hipStream_t s) {
  const TileGeom g = tile_geom(d);
  uint32_t* count = reinterpret_cast<uint32_t*>(ws + L.off_count[set0]);
  uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.off_start);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(ws + L.off_cursor);
  uint32_t* bcur = reinterpret_cast<uint32_t*>(ws + L.off_bcur);
  uint32_t* bcnt = reinterpret_cast<uint32_t*>(ws + L.off_bcnt);
  Rec<RS>* rec = reinterpret_cast<Rec<RS>*>(ws + L.off_rec);
  Rec<RS>* region = reinterpret_cast<Rec<RS>*>(ws + L.off_region);
  Rec<RS>* ovf_rec = reinterpret_cast<Rec<RS>*>(ws + L.off_ovf);
  double* partial = reinterpret_cast<double*>(ws + L.off_partial);
  const uint32_t cap = bucket_cap(n, L.nbuckets);  // <= L.cap
  // knob value 2 of CNPC_TUNE_SORT_FUSED: the Y_lm sums (l = 2, 4) in a pass
  // of their own, which keeps the bucket pass at the register count of the
  // l = 0 sums
  const bool split_sums = sums_lmax >= 2 && tune_value(CNPC_TUNE_SORT_FUSED) == 2;
  const int lm = split_sums ? 0 : (sums_lmax >= 4 ? 4 : (sums_lmax >= 2 ? 2 : 0));
  BucketShape bs = bucket_shape(RS, lm);
  const int ltiles = L.ntiles <= LDS_TILES_MAX ? L.ntiles : 0;
  const bool pack = packs_records(sizeof(T) == 4, RS, g.shift);  // records of the FP32 painter
  const bool packb = pack && L.ntiles <= 65536;                  // bucket records packed too
  auto blds = [&](const BucketShape& b) {
    return bucket_pass_lds(b.per, RS, L.nbuckets, b.nt, ltiles) + (packb ? (size_t)b.nt * b.per * 2 : 0);
  };
  size_t lds = blds(bs);
  if (bs.per == 8 && lds > lds_limit()) {  // many buckets (N >= 1024): 4 per thread
    bs = {BUCKET_NT, 4, false, BUCKET_BLOCKS_MAX};
    lds = blds(bs);
  }
  const int64_t ch = (int64_t)bs.nt * bs.per;
  const unsigned nblk = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + ch - 1) / ch, bs.maxblk));
  if (lds > lds_limit()) {
    set_error("bucket pass: %zu bytes of LDS exceed the workgroup limit", lds);
    return CNPC_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_zero2_u32, dim3(64), dim3(256), 0, s, count, (int64_t)L.ntiles, bcnt,
                     (int64_t)L.nbuckets + 1);
  CNPC_HIP(hipGetLastError());
  SumsArgs sa;
  sa.lmax = sums_lmax;
  sa.boxsize = d->boxsize;
  for (int i = 0; i < 3; ++i) { sa.obs[i] = d->observer[i]; sa.los[i] = d->los[i]; }
  sa.global_los = d->los_mode == CNPC_LOS_GLOBAL;
  BucketArgs ba;
  ba.g = g;
  ba.ntiles = L.ntiles;
  ba.nbuckets = L.nbuckets;
  ba.cap = cap;
  ba.bcnt = bcnt;
  ba.ovf = bcnt + L.nbuckets;
  ba.tcount = count;
  ba.partial = partial;
  ba.pack = packb;
  ba.rkey = reinterpret_cast<uint16_t*>(reinterpret_cast<uint64_t*>(region) + (int64_t)L.nbuckets * cap);
  ba.okey = reinterpret_cast<uint16_t*>(reinterpret_cast<uint64_t*>(ovf_rec) + n);
  kt_begin(CNPC_KT_SORT, s);
  if (lm == 4) launch_bucket_pass<RS, 4>(bs, nblk, lds, pos, w, n, sa, ba, region, ovf_rec, s);
  else if (lm == 2) launch_bucket_pass<RS, 2>(bs, nblk, lds, pos, w, n, sa, ba, region, ovf_rec, s);
  else launch_bucket_pass<RS, 0>(bs, nblk, lds, pos, w, n, sa, ba, region, ovf_rec, s);
  kt_end(CNPC_KT_SORT, s);
  CNPC_HIP(hipGetLastError());
  const int per_bucket = 1 << (3 * g.ls);
  if (split_sums) {
    CountArgs none;
    none.ntiles = 0;
    none.count = nullptr;
    CNPC_TRY(sums_counted(d, pos, w, n, sums_lmax, sums, partial, none, s));
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, count, L.ntiles, per_bucket, start, cursor, bcur);
  } else {
    // tile scan and the column sums of the bucket pass's partials in one launch
    hipLaunchKernelGGL(k_tile_scan_sums, dim3(1 + CNPC_SUMS_LEN), dim3(1024), 0, s, count, L.ntiles, per_bucket,
                       start, cursor, bcur, partial, (int)nblk, sums);
  }
  CNPC_HIP(hipGetLastError());
  // tile pass: one workgroup per region chunk, then OVF_BLOCKS over the overflow
  const int tper = partition_per(RS, per_bucket, 1024);
  if (tper == 0) {
    set_error("tile pass: %d keys do not fit the LDS of a workgroup", per_bucket);
    return CNPC_EINVAL;
  }
  const int64_t tch = (int64_t)1024 * tper;
  const int cpb = (int)((cap + tch - 1) / tch);
  const unsigned tgrid = (unsigned)(L.nbuckets * cpb + OVF_BLOCKS);
  const size_t tlds = partition_lds(tper, RS, per_bucket, 1024);
  kt_begin(CNPC_KT_SORT, s);
  if (packb) {
    const size_t plds = (size_t)1024 * tper * 10 + (size_t)3 * per_bucket * 4 + 64;
    const uint64_t* r64 = reinterpret_cast<const uint64_t*>(region);
    const uint64_t* o64 = reinterpret_cast<const uint64_t*>(ovf_rec);
    uint64_t* out64 = reinterpret_cast<uint64_t*>(rec);
    if (tper == 4)
      hipLaunchKernelGGL((k_tile_pass_packed<4, 1024>), dim3(tgrid), dim3(1024), plds, s, r64, ba.rkey, o64, ba.okey,
                         bcnt, bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, out64);
    else if (tper == 2)
      hipLaunchKernelGGL((k_tile_pass_packed<2, 1024>), dim3(tgrid), dim3(1024), plds, s, r64, ba.rkey, o64, ba.okey,
                         bcnt, bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, out64);
    else
      hipLaunchKernelGGL((k_tile_pass_packed<1, 1024>), dim3(tgrid), dim3(1024), plds, s, r64, ba.rkey, o64, ba.okey,
                         bcnt, bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, out64);
    kt_end(CNPC_KT_SORT, s);
    CNPC_HIP(hipGetLastError());
    return paint_sorted<T, RS>(d, weighted, set0, ws, L, s);
  }
  if (tper == 4)
    hipLaunchKernelGGL((k_tile_pass<RS, 4, 1024>), dim3(tgrid), dim3(1024), tlds, s, region, ovf_rec, bcnt,
                       bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, rec, pack);
  else if (tper == 2)
    hipLaunchKernelGGL((k_tile_pass<RS, 2, 1024>), dim3(tgrid), dim3(1024), tlds, s, region, ovf_rec, bcnt,
                       bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, rec, pack);
  else
    hipLaunchKernelGGL((k_tile_pass<RS, 1, 1024>), dim3(tgrid), dim3(1024), tlds, s, region, ovf_rec, bcnt,
                       bcnt + L.nbuckets, cap, cpb, L.nbuckets, g, cursor, rec, pack);
  kt_end(CNPC_KT_SORT, s);
  CNPC_HIP(hipGetLastError());
  return paint_sorted<T, RS>(d, weighted, set0, ws, L, s);
}

// fused: sums_lmax >= 0 selects the fused bucket pass (catalog sums into
// gs / rs, norms formed after both catalogs); counted: tile counts already taken.
template <typename T>
static cnpc_status paint_t(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                           int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                           const double* norms, T* delta, T* noise, unsigned char* ws,
                           const PaintLayout& L, bool counted, hipStream_t s, int sums_lmax = -1,
                           double* gs = nullptr, double* rs = nullptr, bool fold = true) {
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  const uint32_t* cpos[2] = {gpos, rpos};
  const float* cw[2] = {gw, rw};
  const int64_t cn[2] = {ngal, nran};
  FoldArgs<T> fa;
  fa.n = d->n;
  fa.nt = L.nt;
  fa.nphase = L.nphase;
  fa.nsets = L.nsets;
  for (int c = 0; c < 2; ++c) {
    for (int pw = 0; pw < (weighted ? 2 : 1); ++pw)
      fa.blocks[c + 2 * pw] = reinterpret_cast<T*>(ws + L.off_blocks[c + 2 * pw]);
    double* sums_c = c == 0 ? gs : rs;
    if (sums_lmax >= 0 && cw[c])
      CNPC_TRY((fused_sort_and_paint<T, 4>(d, cpos[c], cw[c], cn[c], c, weighted, sums_lmax, sums_c, ws, L, s)));
    else if (sums_lmax >= 0)
      CNPC_TRY((fused_sort_and_paint<T, 3>(d, cpos[c], nullptr, cn[c], c, weighted, sums_lmax, sums_c, ws, L, s)));
    else if (cw[c])
      CNPC_TRY((sort_and_paint<T, 4>(d, cpos[c], cw[c], cn[c], c, weighted, counted, ws, L, s)));
    else
      CNPC_TRY((sort_and_paint<T, 3>(d, cpos[c], nullptr, cn[c], c, weighted, counted, ws, L, s)));
  }
  if (sums_lmax >= 0) CNPC_TRY(launch_norms(d, gs, rs, ngal, const_cast<double*>(norms), s));
  if (!fold) return CNPC_OK;
  const int z2 = L.nt >= 2 ? 2 : 1;
  const int64_t nb = (int64_t)L.nphase * L.nt * L.nt * (L.nt / z2);
  kt_begin(CNPC_KT_FOLD, s);
  hipLaunchKernelGGL((k_fold_tiles<T>), dim3((unsigned)nb), dim3(256 * z2), 0, s, fa, norms, delta, noise);
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
                           L, false, s);
  return paint_t<float>(d, gpos, gw, ngal, rpos, rw, nran, norms, (float*)delta, (float*)noise, w, L,
                        false, s);
}

bool has_fold_zr2c(const cnpc_mesh_desc* d) {
  return d->interlace && d->n == 256 && fft_register_passes();
}

template <typename T>
static cnpc_status fold_zr2c_t(const cnpc_mesh_desc* d, const PaintLayout& L, unsigned char* ws,
                               const double* norms, cx<T>* dsp, cx<T>* nw1, int m, hipStream_t s) {
  FoldArgs<T> fa;
  fa.n = d->n;
  fa.nt = L.nt;
  fa.nphase = L.nphase;
  fa.nsets = L.nsets;
  for (int k = 0; k < L.nsets; ++k) fa.blocks[k] = reinterpret_cast<T*>(ws + L.off_blocks[k]);
  // one workgroup per (phase, tile column, x node of the tile)
  const int64_t grid = (int64_t)L.nphase * L.nt * L.nt * TILE;
  const size_t lds = sizeof(cx<T>) * (256 + (size_t)16 * FZ_RS);
  CNPC_TRY(ensure_twiddles());
  kt_begin(CNPC_KT_FOLD, s);
  hipLaunchKernelGGL((k_fold_zr2c<T>), dim3((unsigned)grid), dim3(256), lds, s, fa, norms, dsp, d->n / 2, nw1, m);
  kt_end(CNPC_KT_FOLD, s);
  CNPC_HIP(hipGetLastError());
  return CNPC_OK;
}

cnpc_status launch_paint_blocks_zr2c(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw, int64_t ngal,
                                     const uint32_t* rpos, const float* rw, int64_t nran, int sums_lmax,
                                     double* gsums, double* rsums, double* norms, void* dsp, void* nw1, int m,
                                     void* ws, size_t ws_bytes, hipStream_t s) {
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  PaintLayout L = paint_layout(d, ngal, nran, weighted);
  if (ws_bytes < L.total) {
    set_error("paint workspace too small: need %zu bytes, got %zu", L.total, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  if (!has_fold_zr2c(d)) {
    set_error("fused fold and z pass: unsupported mesh");
    return CNPC_EUNSUPPORTED;
  }
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  const bool fused = L.nbuckets > 1 && tune_value(CNPC_TUNE_SORT_FUSED) != 1;
  if (!fused) {
    // sums and tile counts in a pass of their own, norms before the painting
    uint32_t* count0 = reinterpret_cast<uint32_t*>(w + L.off_count[0]);
    uint32_t* count1 = reinterpret_cast<uint32_t*>(w + L.off_count[1]);
    double* partial = reinterpret_cast<double*>(w + L.off_partial);
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count0, (int64_t)L.ntiles);
    hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count1, (int64_t)L.ntiles);
    CNPC_HIP(hipGetLastError());
    CountArgs ca;
    ca.g = tile_geom(d);
    ca.ntiles = L.ntiles;
    ca.count = count0;
    CNPC_TRY(sums_counted(d, gpos, gw, ngal, sums_lmax, gsums, partial, ca, s));
    ca.count = count1;
    CNPC_TRY(sums_counted(d, rpos, rw, nran, sums_lmax, rsums, partial, ca, s));
    CNPC_TRY(launch_norms(d, gsums, rsums, ngal, norms, s));
  }
  const int lm = fused ? sums_lmax : -1;
  if (d->dtype == CNPC_F64) {
    CNPC_TRY(paint_t<double>(d, gpos, gw, ngal, rpos, rw, nran, norms, nullptr, nullptr, w, L, !fused, s, lm,
                             gsums, rsums, false));
    return fold_zr2c_t<double>(d, L, w, norms, (cx<double>*)dsp, (cx<double>*)nw1, m, s);
  }
  CNPC_TRY(paint_t<float>(d, gpos, gw, ngal, rpos, rw, nran, norms, nullptr, nullptr, w, L, !fused, s, lm, gsums,
                          rsums, false));
  return fold_zr2c_t<float>(d, L, w, norms, (cx<float>*)dsp, (cx<float>*)nw1, m, s);
}

cnpc_status launch_paint_fkp(const cnpc_mesh_desc* d, const uint32_t* gpos, const float* gw,
                             int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                             int sums_lmax, double* gsums, double* rsums, double* norms, void* delta,
                             void* noise, void* ws, size_t ws_bytes, hipStream_t s) {
  const bool weighted = (gw != nullptr) || (rw != nullptr);
  PaintLayout L = paint_layout(d, ngal, nran, weighted);
  if (ws_bytes < L.total) {
    set_error("paint workspace too small: need %zu bytes, got %zu", L.total, ws_bytes);
    return CNPC_EWORKSPACE;
  }
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  double* gs_ = gsums ? gsums : reinterpret_cast<double*>(w + L.off_sums);
  double* rs_ = rsums ? rsums : reinterpret_cast<double*>(w + L.off_sums) + CNPC_SUMS_LEN;
  if (L.nbuckets > 1 && tune_value(CNPC_TUNE_SORT_FUSED) != 1) {
    if (d->dtype == CNPC_F64)
      return paint_t<double>(d, gpos, gw, ngal, rpos, rw, nran, norms, (double*)delta, (double*)noise, w, L,
                             false, s, sums_lmax, gs_, rs_);
    return paint_t<float>(d, gpos, gw, ngal, rpos, rw, nran, norms, (float*)delta, (float*)noise, w, L, false,
                          s, sums_lmax, gs_, rs_);
  }
  uint32_t* count0 = reinterpret_cast<uint32_t*>(w + L.off_count[0]);
  uint32_t* count1 = reinterpret_cast<uint32_t*>(w + L.off_count[1]);
  double* partial = reinterpret_cast<double*>(w + L.off_partial);
  double* gs = gsums ? gsums : reinterpret_cast<double*>(w + L.off_sums);
  double* rs = rsums ? rsums : reinterpret_cast<double*>(w + L.off_sums) + CNPC_SUMS_LEN;
  hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count0, (int64_t)L.ntiles);
  hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, s, count1, (int64_t)L.ntiles);
  CNPC_HIP(hipGetLastError());
  CountArgs ca;
  ca.g = tile_geom(d);
  ca.ntiles = L.ntiles;
  ca.count = count0;
  CNPC_TRY(sums_counted(d, gpos, gw, ngal, sums_lmax, gs, partial, ca, s));
  ca.count = count1;
  CNPC_TRY(sums_counted(d, rpos, rw, nran, sums_lmax, rs, partial, ca, s));
  CNPC_TRY(launch_norms(d, gs, rs, ngal, norms, s));
  if (d->dtype == CNPC_F64)
    return paint_t<double>(d, gpos, gw, ngal, rpos, rw, nran, norms, (double*)delta, (double*)noise, w,
                           L, true, s);
  return paint_t<float>(d, gpos, gw, ngal, rpos, rw, nran, norms, (float*)delta, (float*)noise, w, L,
                        true, s);
}

}  // namespace cnpc
