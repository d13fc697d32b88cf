/*
 * cnpc.h -- C ABI of the MI355X (gfx950) FFT clustering-estimator library.
 *
 * Computes the Yamamoto power-spectrum multipoles, the modified high-order
 * multipoles, the Scoccimarro bispectrum multipoles and the compressed TripoSH
 * bispectrum B_l0l with analytic shot noise, following "Efficient estimators
 * for power spectrum and bispectrum multipole measurements" (Xie et al.).
 * Section and equation names below refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All data pointers are DEVICE pointers unless a parameter says "host".
 *    The caller owns every buffer it passes.  Scratch space is passed in as
 *    `ws` / `ws_bytes`, sized by the matching *_workspace_size query.
 *  - Every compute call is asynchronous on `stream` (a hipStream_t, NULL =
 *    default stream), allocates no device memory and does not synchronise;
 *    outputs are valid once the stream has synchronised.  The set-up calls
 *    are the exceptions: cnpc_bispec_plan_create and cnpc_sugi_plan_create
 *    allocate the plan's small device tables (configurations, factors, pair
 *    rows) with blocking copies, and a Scoccimarro plan computes N_T on
 *    `stream` and synchronises it to read them back; cnpc_batch_create
 *    creates streams and events, cnpc_batch_capture a HIP graph,
 *    cnpc_ktimer_start events; the first transform on a device uploads a
 *    16 KiB twiddle table with a blocking copy.  Destroy calls free what
 *    their create call allocated.
 *  - Return value: CNPC_OK (0) or a negative status.  Arguments are validated
 *    on the host before anything is launched; on error nothing is launched and
 *    cnpc_last_error() (thread-local) describes the problem.
 *  - Positions are 3 x uint32 fixed point p = floor(x / L * 2^32), stored
 *    structure-of-arrays: pos[0..n) = x, pos[n..2n) = y, pos[2n..3n) = z.
 *  - Weights w are FP32 (NULL means w = 1 for every particle).
 *  - Real meshes are N^3 values, index (ix * N + iy) * N + iz, node j at x = jH
 *    (H = L/N).  With interlacing a second mesh B (nodes at (j + 1/2) H)
 *    follows mesh A contiguously.
 *  - Full half spectra ("half layout") hold N * N * (N/2) complex values
 *    (re, im interleaved), index (ix * N + iy) * (N/2) + kz, kz = 0..N/2-1.
 *    The kz = N/2 plane is not stored: every estimator zeroes modes with a
 *    Nyquist component.  Wavenumber index n = i for i < N/2, i - N otherwise.
 *  - Band spectra ("band layout", band half-width M, a power of two <= N/2)
 *    hold only modes with |nx|, |ny| < M and 0 <= nz < M:
 *    (2M) * (2M) * M complex values, index (jx * 2M + jy) * M + kz with
 *    n = j for j < M and j - 2M otherwise.  Every binned mode lies in the band
 *    when M > k_max / k_f (k_f = 2 pi / L); cnpc_band_for() returns the
 *    smallest such M.  Forward band transforms fill the n = -M rows; inverse
 *    band transforms read them as zero (they have no +M partner).
 *  - Element type follows desc->dtype: float / float2 (CNPC_F32) or
 *    double / double2 (CNPC_F64).  Shell accumulators, catalog sums,
 *    normalisations and shot-noise terms are always FP64.
 *  - Forward transforms use exp(-i k.x) (the sign of eq. key1); inverse
 *    transforms use exp(+i k.x) and are unnormalised.
 */
#ifndef CNPC_H
#define CNPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cnpc_status;
#define CNPC_OK 0
#define CNPC_EINVAL (-1)       /* invalid argument (null pointer, bad size, ...) */
#define CNPC_EWORKSPACE (-2)   /* workspace smaller than the query returned */
#define CNPC_EHIP (-3)         /* a HIP runtime call failed */
#define CNPC_EUNSUPPORTED (-4) /* valid but not supported (e.g. N > 1024) */

#define CNPC_F32 0
#define CNPC_F64 1
#define CNPC_CIC 2
#define CNPC_TSC 3
#define CNPC_LOS_LOCAL 0  /* xhat = unit vector from the observer to the node */
#define CNPC_LOS_GLOBAL 1 /* xhat = desc->los for every node */

/* Mesh / catalog geometry.  n: power of two in [16, 1024].  observer: used
 * with CNPC_LOS_LOCAL; must lie outside the box.  los: unit vector used with
 * CNPC_LOS_GLOBAL. */
typedef struct {
  int32_t n;
  int32_t assign;    /* CNPC_CIC or CNPC_TSC */
  int32_t interlace; /* 0 or 1 */
  int32_t dtype;     /* CNPC_F32 or CNPC_F64 */
  int32_t los_mode;  /* CNPC_LOS_LOCAL or CNPC_LOS_GLOBAL */
  int32_t reserved;
  double boxsize; /* L */
  double observer[3];
  double los[3];
} cnpc_mesh_desc;

/* k bins: half-open [kmin + b dk, kmin + (b+1) dk), b = 0..nbins-1.  Mode
 * membership is decided on the integer |n|^2 with thresholds
 * T_b = ceil(((kmin + b dk) / k_f)^2) computed in FP64, an edge whose square is
 * within a relative 1e-9 of an integer counting as exactly on it (a reading of
 * the binning mask of the Sugiyama section, whose printed inequalities differ
 * between its equations).  The k = 0 mode and modes with a Nyquist component are excluded.  The top
 * edge must not exceed the Nyquist wavenumber. */
typedef struct {
  double kmin;
  double dk;
  int32_t nbins;
  int32_t reserved;
} cnpc_kbins;

/* ---- catalog sums (sections on the Yamamoto and Scoccimarro estimators) ----
 * Per catalog FP64 sums: [0] sum w, [1] sum w^2, [2] sum w^3, then for
 * (l, m) in (0,0),(2,0),(2,1),(2,2),(4,0),...,(4,4): re, im of
 * sum w^3 y_l^m*(xhat) (Racah-normalised harmonics, xhat from the observer to
 * the particle, or desc->los).  CNPC_SUMS_LEN doubles. */
#define CNPC_NYLM_SUMS 9
#define CNPC_SUMS_LEN (3 + 2 * CNPC_NYLM_SUMS)
size_t cnpc_catalog_sums_workspace_size(void);
cnpc_status cnpc_catalog_sums(const cnpc_mesh_desc* desc, const uint32_t* pos, const float* w,
                              int64_t n, double* sums, void* ws, size_t ws_bytes, void* stream);

/* Normalisations from the galaxy and random sums (under eq. Hand17 and
 * eq. bi_sco; the Sbar terms of eq. Q_ell): CNPC_NORMS_LEN doubles
 *   [0] alpha = sum_g w / sum_r w      [1] nbar = ngal / L^3
 *   [2] I22 = alpha nbar sum_r w^2     [3] I33 = alpha nbar^2 sum_r w^3
 *   [4] N0 = (sum_g w^2 + alpha^2 sum_r w^2) / I22
 *   [5] Sbar = sum_g w^3 - alpha^3 sum_r w^3
 *   [6 + 2q], [7 + 2q]: re, im of Sbar_l^m for the q-th (l, m) listed above
 * Computed on the device (no host synchronisation). */
#define CNPC_NORM_ALPHA 0
#define CNPC_NORM_NBAR 1
#define CNPC_NORM_I22 2
#define CNPC_NORM_I33 3
#define CNPC_NORM_N0 4
#define CNPC_NORM_SBAR 5
#define CNPC_NORM_SBARLM 6
#define CNPC_NORMS_LEN (6 + 2 * CNPC_NYLM_SUMS)
cnpc_status cnpc_norms(const cnpc_mesh_desc* desc, const double* gal_sums, const double* ran_sums,
                       int64_t ngal, double* norms, void* stream);

/* ---- paint: mass assignment of the FKP field (section on modified high-order
 * multipoles, TSC assignment) ----
 * delta = n_g - alpha n_r (weights w) and, when noise != NULL, the shot-noise
 * mesh N = n_g(w^2) + alpha^2 n_r(w^2) (definition of N_l^m under
 * eq. generic_noise).  alpha is read from norms[CNPC_NORM_ALPHA] on the device.
 * CIC: nodes floor(u), floor(u)+1; TSC: nodes floor(u+1/2)+{-1,0,1}, with
 * u = p N / 2^32 (mesh B: u - 1/2).  Outputs are overwritten (not accumulated):
 * delta and noise each hold (1 + interlace) N^3 elements of desc->dtype.
 * Particles are counting-sorted by 16^3-node tiles and accumulated in LDS as
 * integer fixed point (2^-40 units; 2^-21 for unit-weight FP32), so the
 * meshes do not depend on the order of the additions.  Unit-weight FP32
 * meshes of 256^3 and more take the positions truncated to a 2^-17 cell grid
 * inside their tile (8-byte sort records); the FP64 path, weighted catalogs,
 * coarser meshes and the catalog sums use the full 32-bit positions.
 * Workspace: cnpc_paint_workspace_size bytes (an upper bound for weighted and
 * unweighted catalogs), owned by the caller, not retained after the call. */
size_t cnpc_paint_workspace_size(const cnpc_mesh_desc* desc, int64_t ngal, int64_t nran);
cnpc_status cnpc_paint(const cnpc_mesh_desc* desc, const uint32_t* gpos, const float* gw,
                       int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                       const double* norms, void* delta, void* noise, void* ws, size_t ws_bytes,
                       void* stream);
/* cnpc_catalog_sums of both catalogs, cnpc_norms and cnpc_paint in one call:
 * the tile histogram of the sort is taken during the catalog-sum pass, which
 * saves one read of every particle.  sums_lmax (0, 2 or 4): the Y_l^m sums
 * (and Sbar_l^m) are formed for l <= sums_lmax only, the others are zero; the
 * l = 0 sums are always formed.  gal_sums, ran_sums: CNPC_SUMS_LEN device
 * doubles each, or NULL when not wanted; norms: CNPC_NORMS_LEN device doubles
 * (output).  Same meshes and workspace size as cnpc_paint; sums_lmax = 4
 * gives the sums of cnpc_catalog_sums bit for bit. */
cnpc_status cnpc_paint_fkp(const cnpc_mesh_desc* desc, const uint32_t* gpos, const float* gw,
                           int64_t ngal, const uint32_t* rpos, const float* rw, int64_t nran,
                           int32_t sums_lmax, double* gal_sums, double* ran_sums, double* norms,
                           void* delta, void* noise, void* ws, size_t ws_bytes, void* stream);

/* ---- fft: batched 3-D real transforms (all hot-path transforms) ----
 * Full r2c: `batch` real meshes -> half-layout spectra.  Full c2r: half-layout
 * spectra (kz = N/2 plane taken as zero) -> real meshes.  Band r2c: real
 * meshes -> band-layout spectra (half-width M); band c2r: band spectra (modes
 * outside the band taken as zero) -> real meshes.  in and out must not
 * overlap; out of a c2r may alias nothing else.  Scratch: ws of
 * cnpc_fft_workspace_size bytes. */
size_t cnpc_fft_workspace_size(const cnpc_mesh_desc* desc, int32_t batch, int32_t band);
cnpc_status cnpc_fft_r2c(const cnpc_mesh_desc* desc, int32_t batch, int32_t band, const void* in,
                         void* out, void* ws, size_t ws_bytes, void* stream);
cnpc_status cnpc_fft_c2r(const cnpc_mesh_desc* desc, int32_t batch, int32_t band, const void* in,
                         void* out, void* ws, size_t ws_bytes, void* stream);
int32_t cnpc_band_for(const cnpc_mesh_desc* desc, double kmax);

/* ---- interlacing and de-aliasing (design reading; not in the paper) ----
 * From the painted meshes A (and B): D(k) = 1/2 [D_A(k) + exp(-i k.(1,1,1)H/2) D_B(k)]
 * with every Nyquist-component mode zeroed (without interlacing D = D_A).
 * Writes D in band layout (half-width `band`, the n = -band rows included) to
 * spec_band and, when
 * delta_int != NULL, the de-aliased real mesh IDFT(D) / N^3 (without
 * interlacing: a copy of A). */
size_t cnpc_deinterlace_workspace_size(const cnpc_mesh_desc* desc);
cnpc_status cnpc_deinterlace(const cnpc_mesh_desc* desc, int32_t band, const void* meshes,
                             void* spec_band, void* delta_int, void* ws, size_t ws_bytes,
                             void* stream);

/* ---- painting with de-interlacing (cnpc_paint_fkp followed by cnpc_deinterlace
 * of the delta mesh with delta_int and of the N mesh, in one call) ----
 * Interlaced meshes of side 256 (register FFT passes, the default) only;
 * other meshes return CNPC_EUNSUPPORTED.  The tile sums of the painting are
 * taken inside the z passes of the two de-interlacing transforms, so the
 * delta and N meshes are never stored.  Arguments as in cnpc_paint_fkp and
 * cnpc_deinterlace; outputs (device): the catalog sums (optional), norms, the
 * band spectrum D and delta_int (N^3 reals) of delta, the band spectrum of N.
 * Workspace: cnpc_paint_deinterlace_workspace_size (weighted: 1 if weights are
 * given).  Results equal the two-step form within FP rounding. */
size_t cnpc_paint_deinterlace_workspace_size(const cnpc_mesh_desc* desc, int64_t ngal, int64_t nran,
                                             int32_t weighted, int32_t band);
cnpc_status cnpc_paint_deinterlace(const cnpc_mesh_desc* desc, int32_t band, const uint32_t* gal_pos,
                                   const float* gal_w, int64_t ngal, const uint32_t* ran_pos, const float* ran_w,
                                   int64_t nran, int32_t sums_lmax, double* gal_sums, double* ran_sums,
                                   double* norms, void* spec_band, void* delta_int, void* noise_spec_band,
                                   void* ws, size_t ws_bytes, void* stream);

/* ---- ylm_fields: Y_lm-weighted real fields (eq. key1, eq. hand, eq. F_lm_SIC) ----
 * Materialised form: out = (2l+1) real meshes delta(x) * [Re y_l^0, Re y_l^1,
 * Im y_l^1, ..., Re y_l^l, Im y_l^l](xhat) (Racah-normalised, m >= 0 only; the
 * m < 0 fields follow from the conjugation symmetry).  l in 0..4. */
cnpc_status cnpc_ylm_fields(const cnpc_mesh_desc* desc, int32_t ell, const void* delta, void* out,
                            void* stream);
/* Fused form: the same fields for every l in ells[0..nells) (host array,
 * each l in {1,2,3,4}) transformed straight to band spectra without being
 * materialised: out holds sum(2l+1) band spectra in that order. */
size_t cnpc_ylm_r2c_workspace_size(const cnpc_mesh_desc* desc, int32_t nfields, int32_t band);
cnpc_status cnpc_ylm_r2c(const cnpc_mesh_desc* desc, int32_t band, int32_t nells,
                         const int32_t* ells, const void* delta, void* out, void* ws,
                         size_t ws_bytes, void* stream);

/* ---- F_l assembly (eq. hand with eq. F_lm_SIC on the r2c half spectrum) ----
 * F_l(k) = [c_0 A_0 + 2 sum_{m>=1} (c_m A_m + s_m B_m)](k) / W(k), with
 * c_m + i s_m = y_l^m(khat), A_m, B_m the band spectra of the Re / Im fields,
 * W(k) = prod_i sinc(pi n_i / N)^p (eq. compensation), F_l(0) = 0.
 * l = 0: F_0 = D / W from the de-interlaced spectrum alone (ylm may be NULL).
 * Output: one band spectrum. */
cnpc_status cnpc_assemble_F(const cnpc_mesh_desc* desc, int32_t band, int32_t ell,
                            const void* spec0, const void* ylm, void* F_out, void* stream);

/* ---- bin_pk: shell means (eqs. Hand17, pk_final, Pllp; eqs. Q_ell, H_ell) ----
 * For each of npairs products (a, b) (host arrays pa, pb of band-spectrum
 * pointers, device), accumulates in FP64 over the modes of every bin
 *   sum Re F_a(k) F_b(k)^*        (Hermitian half-grid weights 1 / 2)
 * and, per bin, N_mode (int64, exact) and sum |k|.  With self_ells != NULL
 * (host, nself entries), also the shell mean of the self-pair term
 *   s_l(k) = < sum_m y_l^m(khat) Sbar_l^m C(k) / W(k)^2 >
 * where C is the alias sum of the squared window (interlaced: half the sum of
 * the plain and the alternating image sums), reading Sbar_l^m from norms.
 * Output (device, FP64): means[npairs][nbins] = shell means, selfterm[nself][nbins],
 * nmodes[nbins], keff[nbins] (mean |k|).  No normalisation is applied here.
 * Limits: nbins <= 128, npairs <= 16, nself <= 4 with self_ells in {0, 2, 4}.
 * pa, pb, self_ells are host arrays; the spectra they point to are device
 * band spectra (half-width `band`). */
size_t cnpc_bin_pk_workspace_size(const cnpc_kbins* bins, int32_t npairs, int32_t nself);
cnpc_status cnpc_bin_pk(const cnpc_mesh_desc* desc, const cnpc_kbins* bins, int32_t band,
                        int32_t npairs, const void* const* pa, const void* const* pb,
                        int32_t nself, const int32_t* self_ells, const double* norms,
                        double* means, double* selfterm, int64_t* nmodes, double* keff,
                        void* ws, size_t ws_bytes, void* stream);

/* cnpc_bin_pk without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, outputs and limits as cnpc_bin_pk;
 * the FP64 shell accumulators live in a static device array of
 * 128 * (16 + 4 + 1) doubles (21.5 KiB, the largest binning cnpc_bin_pk
 * accepts), one per GPU, held until the process ends; nbins * (npairs + nself
 * + 1) above that is rejected with CNPC_EINVAL.  No call allocates or frees
 * memory.  Every call on a GPU uses that GPU's one array (cleared by the call
 * itself), so calls that overlap on one GPU, on any streams, race: serialise
 * them.  The stream must belong to the current device. */
cnpc_status cnpc_bin_pk_noalloc(const cnpc_mesh_desc* desc, const cnpc_kbins* bins, int32_t band,
                                int32_t npairs, const void* const* pa, const void* const* pb,
                                int32_t nself, const int32_t* self_ells, const double* norms,
                                double* means, double* selfterm, int64_t* nmodes, double* keff,
                                void* stream);

/* Shell means of Im F_a(k) F_b(k)^* (odd multipoles: the imaginary-part form
 * of eq. pk_final).  Same arguments, limits and workspace as cnpc_bin_pk with
 * no self terms; for anti-Hermitian products (F_0 F_l^*, l odd) the half-grid
 * weights apply unchanged. */
cnpc_status cnpc_bin_pk_im(const cnpc_mesh_desc* desc, const cnpc_kbins* bins, int32_t band,
                           int32_t npairs, const void* const* pa, const void* const* pb,
                           double* means, int64_t* nmodes, double* keff, void* ws, size_t ws_bytes,
                           void* stream);

/* One multipole from its shell mean: out = (2l+1) mean / I22 - delta_l0 N0
 * (eq. Hand17; odd l with the Im mean of cnpc_bin_pk_im; no shot noise for
 * l > 0).  l in [0, 8]; mean, norms, out device, nbins values. */
cnpc_status cnpc_pk_multipole(const cnpc_kbins* bins, int32_t ell, const double* mean,
                              const double* norms, double* out, void* stream);

/* Normalisations of the cross multipoles of two tracers A, B (the toolkit
 * section's core functionality: auto and cross correlations of several
 * tracers; the paper gives no normalisation, this is the library's reading):
 * the norms of A with I22 = sqrt(I22_A I22_B) and N0 = 0 (distinct samples
 * share no galaxy).  All device, CNPC_NORMS_LEN
 * doubles. */
cnpc_status cnpc_cross_norms(const double* norms_a, const double* norms_b, double* norms_out,
                             void* stream);

/* Yamamoto multipoles from the shell means (eq. Hand17 / eq. Pllp / eq. Plnew):
 * P_l = (2l+1)/I22 <Re F_0 F_l*> - delta_l0 N0, P_ll' = (2(l+l')+1)/I22
 * <Re F_l F_l'*> - N_ll' (N_22 = 9 N0/5, N_44 = 17 N0/9, N_42 = 0), and
 * P_4b, P_6b, P_8b.  means_* are the bin_pk outputs for the listed products
 * (NULL when not wanted).  out: [P0, P2, P4, P22, P42, P44, P4b, P6b, P8b][nbins]. */
cnpc_status cnpc_pk_finalize(const cnpc_kbins* bins, const double* mean00, const double* mean02,
                             const double* mean04, const double* mean22, const double* mean42,
                             const double* mean44, const double* norms, double* out, void* stream);

/* ---- bispectrum (eq. bi_sco; eq. new_bispec for B_l0l) ----
 * Shell fields X_i^(l)(x) = sum_{q in bin i} F_l(q) exp(i q.x) by band c2r,
 * G_l = sum_{all q} F_l(q) exp(i q.x), then the grid contraction
 *   C[(a,b), c] = sum_x X_a^(0) X_b^(0) Y_c,  a <= b,
 * with columns Y = [X^(0) shells, X^(l) shells (Scoccimarro, l > 0), G_l
 * (TripoSH)], cast as a GEMM over grid points.  Then
 *   B_l(i; j, k)   = (2l+1)/I33 C / (G^3 N_T) - N^(l)        (Scoccimarro)
 *   BB_l0l(i, j)   = (2l+1)/I33 C / (G^3 N_i N_j) - N_l0l    (TripoSH)
 * The fields and the sum over x live on a G^3 grid (cnpc_bispec_grid), the
 * smallest power of two >= 2M with G > c1 + c2 + c3, where c is the largest
 * |wavevector component| a field holds (shells: below the top bin edge; the
 * unfiltered TripoSH field: M - 1), capped at the mesh size N.  Below N this
 * sum over x has no aliased (q1 + q2 + q3 = G) terms, so it equals G^3 times
 * the sum over exactly closed triangles, as the N^3 sum does.
 * with the analytic shot noise of the shot-noise section (Lemma 1 special
 * case eq. I_l0l, Lemma 2 / eq. g_ell, eqs. Q_ell, H_ell).  Configurations:
 * Scoccimarro l = 0: i <= j <= k; l > 0: any i, j <= k; all closed
 * (largest index <= sum of the other two) with N_T > 0; TripoSH: i <= j.
 * precision: CNPC_PREC_F64 / CNPC_PREC_F32 (VALU contraction in the field
 * type) or CNPC_PREC_BF16X3 (split-BF16 hi+lo MFMA, FP32 accumulation inside a
 * tile, FP64 across tiles; FP32 fields only).
 * See cnpc_bispec_plan for the host-side configuration tables. */
#define CNPC_PREC_F64 0
#define CNPC_PREC_F32 1
#define CNPC_PREC_BF16X3 2
#define CNPC_EST_SCOCCIMARRO 0
#define CNPC_EST_TRIPOSH 1
#define CNPC_EST_SUGIYAMA 2 /* plans of cnpc_sugi_plan_create only */

typedef struct cnpc_bispec_plan cnpc_bispec_plan;
/* Creates the plan (host tables: configurations, triangle counts N_T computed
 * once in FP64 from shell indicator fields on the device, g_l(t) by FP64
 * Gauss-Legendre, alias sums).  Synchronises `stream`.  ws: scratch of
 * cnpc_bispec_workspace_size bytes for the N_T computation and later calls. */
cnpc_status cnpc_bispec_plan_create(cnpc_bispec_plan** plan, const cnpc_mesh_desc* desc,
                                    const cnpc_kbins* bins, int32_t estimator, int32_t ell,
                                    int32_t precision, void* ws, size_t ws_bytes, void* stream);
void cnpc_bispec_plan_destroy(cnpc_bispec_plan* plan);
int32_t cnpc_bispec_nconfigs(const cnpc_bispec_plan* plan);
/* Host copy of the configurations (3 ints each: i, j, k; TripoSH k = -1) and N_T. */
cnpc_status cnpc_bispec_configs(const cnpc_bispec_plan* plan, int32_t* ijk, int64_t* ntri);
size_t cnpc_bispec_workspace_size(const cnpc_mesh_desc* desc, const cnpc_kbins* bins,
                                  int32_t estimator, int32_t ell);
/* F0, Fl: band spectra (half-width cnpc_bispec_band) of F_0 and F_l.
 * noise_means: device FP64 [4][nbins_ext] rows (Q_l, H_l raw shell means
 * <Re F_l N*>, <Re F_0 F_l^N*> and the self term s_l, then N_mode of the
 * extended binning) from cnpc_bin_pk on the extended binning of
 * cnpc_bispec_ext_bins (NULL: no shot noise).  Outputs (device FP64, one value
 * per configuration): raw estimator, shot noise, shot-subtracted estimator. */
int32_t cnpc_bispec_band(const cnpc_bispec_plan* plan);
/* Side G of the grid the shell fields and the contraction use (<= N). */
int32_t cnpc_bispec_grid(const cnpc_bispec_plan* plan);
cnpc_status cnpc_bispec_ext_bins(const cnpc_bispec_plan* plan, cnpc_kbins* ext);
cnpc_status cnpc_bispectrum(const cnpc_bispec_plan* plan, const void* F0, const void* Fl,
                            const double* noise_means, const double* norms, double* raw,
                            double* shot, double* value, void* ws, size_t ws_bytes, void* stream);

/* ---- Sugiyama bispectrum multipoles B_l1l2L (section "Sugiyama estimator":
 * eq. sugi_estimator with eq. F_and_G, the pairing of eq. sym_sugi into
 * eta Re[...]; shot noise of eqs. S3_sugi_new, q_ells and sugi_shot) ----
 *   F_l^m(x; k) = 1/N_k sum_{q in shell k} e^{iq.x} y_l^m*(qhat) F_0(q)
 *   G_L^M(x)    = sum_q e^{iq.x} FFT[delta y_L^M*(xhat)](q) / W(q)
 *   B(k_i, k_j) = H N / I33 sum_{paired (m1, m2, M)} eta (l1 l2 L; m1 m2 M)
 *                 Re 1/G^3 sum_x F_l1^m1(x; k_i) F_l2^m2(x; k_j) G_L^M(x)
 * with y the Racah-normalised harmonics, H = (l1 l2 L; 0 0 0),
 * N = (2l1+1)(2l2+1)(2L+1); the pairs (m1, m2, M), (-m1, -m2, -M) are taken
 * once (M < 0, or M = 0 with m1 <= 0), eta = 2 except (0, 0, 0).  Every
 * field is a real c2r on the plan's grid: F_l^m = c2r[Phi F_0 Re y] +
 * i c2r[Phi F_0 (-Im y)], G_L^M from the Y_L^M r2c spectra of delta; each
 * sub-configuration is up to four shell-pair contractions.
 * Shot noise: delta_l10 delta_l20 delta_L0 Sbar + delta_l1L delta_l20 (2L+1)
 * H_L(k_i) + delta_l2L delta_l10 (2L+1) H_L(k_j) + H N sum_c q(k_i, k_j, k_c)
 * (N_c/k_c) Q_L(k_c) / sum_c N_c/k_c, all over I33, with q of eq. q_ells
 * (Racah-normalised associated Legendre functions, cosines of the closed
 * triangle of bin centres) and c over the bins |i-j| .. i+j.
 * cnpc_sugi_plan_create: l1, l2 in [0, 4] with l1 + l2 even, L in {0, 2, 4},
 * the triangle rule;
 * kmin = 0 and (2 nbins - 1) dk below Nyquist; precision as for
 * cnpc_bispec_plan_create, split BF16 for at most 22 shells.  Destroy with
 * cnpc_bispec_plan_destroy; cnpc_bispec_band / _grid / _ext_bins /
 * _nconfigs (nbins^2, every (i, j)) apply.
 * cnpc_sugiyama: F0 the band spectrum of F_0 (cnpc_assemble_F, l = 0, at the
 * plan's band); ylm the 2L+1 band spectra of cnpc_ylm_r2c for l = L of the
 * de-interlaced delta (NULL when L = 0); noise_means the Q_L, H_L, s_L rows
 * of cnpc_bin_pk on the plan's extended bins (pairs (F_L, N_0), (F_0, F_L^N),
 * self term L), or NULL for no shot noise; raw, shot, value: nbins x nbins
 * device FP64, row i = k_1 bin.  ws: cnpc_sugi_workspace_size bytes.  Errors:
 * CNPC_EINVAL (arguments, a plan of another estimator), CNPC_EWORKSPACE. */
/* cnpc_sugiyama_fft_noise: as cnpc_sugiyama, with the i = j != k noise term by
 * the FFT method (the reference of the section validating the analytic
 * noise): H N / I33 sum eta (l1 l2 L; m1 m2 M) Re 1/G^3 sum_x Y_l1^m1(x; k_i)
 * Y_l2^m2(x; k_j) P_L^M(x) / (N_i N_j), Y the harmonic shell indicators
 * c2r[Phi conj(y)] and P_L^M = c2r[(FFT[delta conj(y_L^M)] / W) conj(N_0) / W
 * - Sbar_L^M C / W^2]
 * (zero at q = 0 and on Nyquist-component modes).  FN0: band spectrum of N_0
 * (cnpc_assemble_F of the N mesh, l = 0); noise_means required (for the H_L
 * terms).  A second pass over the sub-configurations: about twice the cost. */
/* Host utilities of the tripolar basis (no device work):
 * cnpc_tripolar_real_coeffs: the coefficients A^{n1 n2 N}_{l1 l2 L} of the
 * basis in real spherical harmonics (appendix on the real decomposition of
 * bipolar and tripolar bases: 1/H sum_{m1 m2 M} U_m1n1 U_m2n2 U_MN
 * (l1 l2 L; m1 m2 M), U the inverse of the real-harmonic matrix of the
 * spherical-harmonics appendix), written to coeffs[(n1+l1)][(n2+l2)][(N+L)]
 * when coeffs is not NULL (host array of (2l1+1)(2l2+1)(2L+1) doubles), and
 * their number of non-zero entries to *nonzero.  l in [0, 8], triangle rule,
 * even l1 + l2 + L; CNPC_EINVAL otherwise.
 * cnpc_sugi_paired_count: the number of paired complex sub-configurations
 * (m1, m2, M) with a non-zero 3j symbol (what cnpc_sugiyama evaluates before
 * the l1 = l2 reductions); -1 for l outside [0, 8]. */
cnpc_status cnpc_tripolar_real_coeffs(int32_t l1, int32_t l2, int32_t L, double* coeffs, int32_t* nonzero);
int32_t cnpc_sugi_paired_count(int32_t l1, int32_t l2, int32_t L);
size_t cnpc_sugi_workspace_size(const cnpc_mesh_desc* desc, const cnpc_kbins* bins);
cnpc_status cnpc_sugi_plan_create(cnpc_bispec_plan** plan, const cnpc_mesh_desc* desc, const cnpc_kbins* bins,
                                  int32_t l1, int32_t l2, int32_t L, int32_t precision);
cnpc_status cnpc_sugiyama(const cnpc_bispec_plan* plan, const void* F0, const void* ylm,
                          const double* noise_means, const double* norms, double* raw, double* shot,
                          double* value, void* ws, size_t ws_bytes, void* stream);
cnpc_status cnpc_sugiyama_fft_noise(const cnpc_bispec_plan* plan, const void* F0, const void* ylm,
                                    const void* FN0, const double* noise_means, const double* norms,
                                    double* raw, double* shot, double* value, void* ws, size_t ws_bytes,
                                    void* stream);

/* ---- FFT-method shot noise of the TripoSH BB_l0l (the reference method of
 * the section validating the analytic shot noise, applied to the i = j != k
 * term that the new estimator's shot-noise subsection derives) ----
 * The i = j != k term (the two l = 0 legs on one particle) becomes exact:
 *   (2l+1)/I33 T(i, j) / (N_i N_j),
 *   T(i, j) = sum_{q1 in shell i, q2 in shell j} Re P(q1 + q2),
 *   P(q) = F_l(q) N(q)^* - s_l(q)   (s_l(q): the per-mode self-pair term),
 * with P(0) = 0 and P = 0 on modes with a Nyquist component, computed as the
 * contraction sum_x I_i I_j p of the shell indicator fields I_b = c2r[Phi_b]
 * with p = c2r[P] on the plan's grid (no thin-shell step).  The other terms
 * are those of cnpc_bispectrum.
 * cnpc_bispec_indicator_bytes: size of the indicator fields (nbins fields of
 * G^3 values in the plan's field type; 0 for a Scoccimarro plan).
 * cnpc_bispec_indicators: fills them (caller-owned device buffer, computed
 * once per plan and read-only afterwards; ws as for cnpc_bispectrum).
 * cnpc_bispectrum_fft_noise: cnpc_bispectrum of a TripoSH plan with that
 * term exact; FN0 is the band spectrum of F_0 of the N mesh (as F0), ind the
 * filled indicator fields; noise_means as for cnpc_bispectrum (required).
 * Costs a second contraction, one more band c2r and a copy of the indicators
 * into ws.  Errors: CNPC_EINVAL for a Scoccimarro plan or a null pointer,
 * CNPC_EWORKSPACE for a short ws. */
size_t cnpc_bispec_indicator_bytes(const cnpc_bispec_plan* plan);
cnpc_status cnpc_bispec_indicators(const cnpc_bispec_plan* plan, void* ind, void* ws, size_t ws_bytes,
                                   void* stream);
cnpc_status cnpc_bispectrum_fft_noise(const cnpc_bispec_plan* plan, const void* F0, const void* Fl,
                                      const void* FN0, const void* ind, const double* noise_means,
                                      const double* norms, double* raw, double* shot, double* value,
                                      void* ws, size_t ws_bytes, void* stream);

/* ---- batched measurement (the 64-mock workload of P_l and B_0) ----
 * A batch runs many catalog pairs through the whole hot path: catalog sums,
 * painting (cnpc_paint_fkp), de-interlacing of delta and N, the Y_lm r2c
 * transforms of the l > 0 multipoles in ells, F_l assembly, the shell means of
 * F_0 F_l^* and F_0 N^* with the l = 0 self term, P_l (cnpc_pk_finalize rows)
 * and the Scoccimarro B_0 of plan with its analytic shot noise (cnpc_bispectrum
 * rows) -- the steps of the single-catalog entry points, in their order, with
 * two hand-overs of its own on FP32 256^3 meshes: the de-aliased mesh stays as
 * z half spectra for the Y_lm pass (never stored as a real mesh), and the Y_lm
 * row coefficients are formed once per run (results equal to FP32 rounding).
 * Catalog i runs on batch stream i mod nstreams; each stream owns a
 * slab of the caller's workspace for its intermediates, so catalogs on
 * different streams overlap.
 * cnpc_batch_create: plan must be a Scoccimarro l = 0 plan made for desc and
 * bins; ells: 1 to 3 distinct values of {0, 2, 4}, including 0; nstreams in
 * [1, 16]; max_ngal / max_nran bound every later catalog (they size the
 * painting scratch).  The batch owns its streams (default priority), events
 * and a captured graph; it keeps a pointer to plan, which must outlive it.
 * cnpc_batch_workspace_size: bytes of device workspace a run needs (one slab
 * per stream, and ahead of them the FP32 Y_lm row-coefficient table that every
 * catalog of a run shares, formed on `stream` before the batch streams fork).
 * cnpc_batch_run: enqueues ncat catalogs.  Host arrays of ncat device
 * pointers: gpos / rpos (3 x n uint32 positions), pk_out (9 x nbins FP64, the
 * cnpc_pk_finalize rows), bk_out (3 x nconf FP64: raw, shot, value); host
 * arrays ngal / nran; gw / rw: NULL, or arrays of per-catalog FP32 weight
 * pointers (NULL entries: unit weights).  The batch streams wait for the work
 * already on `stream`, and `stream` waits for them at the end.
 * cnpc_batch_capture: captures the same enqueue into a HIP graph held by the
 * batch (replacing an earlier one); nothing runs.  Every pointer is baked
 * into the graph: inputs, outputs and ws must stay allocated, at the same
 * addresses, for as long as the graph is replayed (refill the inputs in place
 * to measure other catalogs of the same sizes).
 * cnpc_batch_replay: launches the captured graph on `stream`.
 * Calls on one batch must not overlap (they share its streams, events and
 * workspace slabs).  Errors: CNPC_EINVAL (arguments, sizes above the maxima,
 * replay before capture), CNPC_EWORKSPACE, CNPC_EHIP. */
typedef struct cnpc_batch cnpc_batch;
cnpc_status cnpc_batch_create(cnpc_batch** batch, const cnpc_mesh_desc* desc, const cnpc_kbins* bins,
                              const cnpc_bispec_plan* plan, int32_t nells, const int32_t* ells,
                              int32_t nstreams, int64_t max_ngal, int64_t max_nran);
size_t cnpc_batch_workspace_size(const cnpc_batch* batch);
cnpc_status cnpc_batch_run(cnpc_batch* batch, int32_t ncat, const uint32_t* const* gpos,
                           const float* const* gw, const int64_t* ngal, const uint32_t* const* rpos,
                           const float* const* rw, const int64_t* nran, double* const* pk_out,
                           double* const* bk_out, void* ws, size_t ws_bytes, void* stream);
cnpc_status cnpc_batch_capture(cnpc_batch* batch, int32_t ncat, const uint32_t* const* gpos,
                               const float* const* gw, const int64_t* ngal, const uint32_t* const* rpos,
                               const float* const* rw, const int64_t* nran, double* const* pk_out,
                               double* const* bk_out, void* ws, size_t ws_bytes);
cnpc_status cnpc_batch_replay(cnpc_batch* batch, void* stream);
void cnpc_batch_destroy(cnpc_batch* batch);

/* ---- kernel timer (measurement hook for benchmarks and profilers) ----
 * While started, every launch of a kernel class selected by class_mask (bit
 * 1 << class) is bracketed by HIP events recorded on its launch stream (at
 * most max_launches launches in total; later ones are not timed).
 * cnpc_ktimer_stop synchronises those events and writes, per class (arrays of
 * 16), the summed kernel time in ms and the number of timed launches.  Not for
 * use under stream capture.  Host-side state: one timer per process. */
#define CNPC_KT_PAINT 1    /* tile accumulation */
#define CNPC_KT_SORT 2     /* tile counting (standalone paint) + bucket / tile scatter */
#define CNPC_KT_FOLD 3     /* block fold into meshes */
#define CNPC_KT_ZR2C 4     /* z-row r2c passes (plain and Y_lm prologue) */
#define CNPC_KT_COL 5      /* x / y column passes */
#define CNPC_KT_ZC2R 6     /* z-row c2r passes */
#define CNPC_KT_CONTRACT 7 /* bispectrum grid contraction */
#define CNPC_KT_BIN 8      /* shell binning */
#define CNPC_KT_SUMS 9     /* catalog sums */
cnpc_status cnpc_ktimer_start(uint32_t class_mask, int32_t max_launches);
cnpc_status cnpc_ktimer_stop(double* ms_per_class, int64_t* launches_per_class);

/* ---- tuning knobs (read by an autotuner; results within each kernel's
 * tolerance whatever the setting, bit-identical paint and binning) ----
 * Process-wide launch choices, read when a call enqueues its kernels (a
 * captured graph keeps the choices made during capture).  Value 0 restores the
 * library's own choice; a value that does not fit a launch (LDS, tile counts)
 * falls back to that choice for that launch.
 *   CNPC_TUNE_FFT_PASSES   1: LDS Stockham passes only; 0: register passes for
 *                          N = 64, 128, 256, 512 where the tile divides.
 *   CNPC_TUNE_FFT_COL_W    columns per workgroup of the LDS column passes
 *                          (power of two 1..64).
 *   CNPC_TUNE_CONTRACT_KG  point groups per contraction workgroup (1, 2, 4).
 *   CNPC_TUNE_SORT_PER     particles per thread of the sort scatter (1, 2, 4).
 *   CNPC_TUNE_SORT_THREADS threads per sort-scatter workgroup (512, 1024).
 *   CNPC_TUNE_SORT_FUSED   cnpc_paint_fkp on meshes of more than one tile
 *                          bucket: 0 (default) takes the catalog sums, the
 *                          tile histogram and the first sort step in one read
 *                          of each catalog; 1 takes the sums and histogram in
 *                          a read of their own; 2 keeps the histogram and the
 *                          l = 0 sums in the first sort step and takes the
 *                          Y_lm sums (l = 2, 4) in a read of their own
 *                          (identical meshes up to the rounding of alpha,
 *                          sums equal to a few ulp).
 *   CNPC_TUNE_FOLD_FUSED   cnpc_paint_deinterlace and the batch runner: 0
 *                          (default) sums the tile blocks inside the z passes
 *                          of the de-interlacing transforms; 1 writes the
 *                          delta and N meshes and transforms them.
 *   CNPC_TUNE_BUCKET       shape of the first sort step of unweighted catalogs
 *                          (0: 1024 threads x 8 particles on one workgroup per
 *                          CU with the l = 0 sums, x 4 with Y_lm sums; 1: 1024
 *                          x 2 with the next chunk loaded during the current
 *                          one; 2: 512 x 4, likewise; 3: 1024 x 4 on two
 *                          workgroups per CU).
 *   CNPC_TUNE_YLM_BASIS    FP32 Y_lm z passes of bands kz < 4 R (N = R^2 of
 *                          the register passes): 0 (default) transforms
 *                          delta R^-L r_z^j, j = 0..L, per parity class of l
 *                          (L its largest l) and forms every field of the
 *                          class from these L + 1 spectra (5 for l = 2, 4);
 *                          1 transforms each field (2l + 1 per l).
 *   CNPC_TUNE_SHELL_FUSED  split-BF16 bispectrum contraction on a 128^3 grid
 *                          (at most 24 fields, 128 shell pairs, 32 columns):
 *                          0 (default) runs the shells' c2r z pass inside the
 *                          contraction, from their z half spectra; 1 writes
 *                          the real shell fields first.
 * cnpc_tune_set rejects unknown knobs and values outside those ranges;
 * cnpc_tune_get returns the current value (-1 for an unknown knob). */
#define CNPC_TUNE_FFT_PASSES 0
#define CNPC_TUNE_FFT_COL_W 1
#define CNPC_TUNE_CONTRACT_KG 2
#define CNPC_TUNE_SORT_PER 3
#define CNPC_TUNE_SORT_THREADS 4
#define CNPC_TUNE_SORT_FUSED 5
#define CNPC_TUNE_FOLD_FUSED 6
#define CNPC_TUNE_BUCKET 7
#define CNPC_TUNE_YLM_BASIS 8
#define CNPC_TUNE_SHELL_FUSED 9
#define CNPC_TUNE_COUNT 10
cnpc_status cnpc_tune_set(int32_t knob, int32_t value);
int32_t cnpc_tune_get(int32_t knob);

/* Last error message of the calling thread ("" when none). */
const char* cnpc_last_error(void);
/* Library version string. */
const char* cnpc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CNPC_H */
