/*
 * ttm.h -- C ABI of the MI355X (gfx950) tensorial template matching engine.
 *
 * Method: Martinez-Sanchez et al., "Tensorial template matching for fast
 * cross-correlation with rotations and its application for tomography"
 * (arXiv 2408.02398).  The library computes, on one GPU,
 *
 *   g      = h * f                         prefilter (Sec. 2, operator S)
 *   w(x)   = 1/sqrt(local masked variance)  (Eq. norm_f)
 *   C_a(x) = w(x) (g * T_a)(x)             tensor field, one FFT correlation
 *                                          per independent component a (Eq. tcc, Alg. 2)
 *   c(x)   = ||C(x)||_F                    position score (Sec. 3.2)
 *   lambda(x), u(x)                        dominant eigenpair of C(x) by SS-HOPM (Sec. 3.1)
 *   peaks                                  P best scores >= 2r apart (Sec. 3.4)
 *
 * and the one-time tensor template T_a (Eq. tt, Alg. 1) with its spectra.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Volumes are float32, layout [z][y][x] with x fastest; vectors are (x, y, z).
 * - Degree n is even (Sec. 3.1: the orientation theorem needs even n), 0 <= n <= 8.
 * - d' = 3: components are indexed by alpha = (ax, ay, az), |alpha| = n, in
 *   graded-lex order (descending ax, then descending ay); K = (n+1)(n+2)/2.
 *   Component alpha holds the full-tensor entry, so ||C||_F^2 = sum mu_a C_a^2
 *   with mu_a = n!/(ax! ay! az!).  d' = 4 (the paper's quaternion form,
 *   K = binom(n+3,3), alpha = (aw, ax, ay, az) in graded-lex order) is
 *   accepted by every entry point; its orientation is a unit quaternion
 *   (w, x, y, z), 4 floats per voxel, from the multistart search at degree
 *   2..6, or from the learned start at degree 2 and 4.
 * - Template: cubic L^3, centre c = L/2 (integer division) on every axis,
 *   binary ball mask m(p) = [|p - c|^2 <= r^2].
 * - Valid region of a volume of extent D along an axis: voxels x with
 *   c <= x <= D - L + c (the whole template window lies inside the volume).
 *   Full-size output maps are 0 outside it.
 * - Every buffer argument is caller-owned.  Pointers documented "device"
 *   must be device memory on the context's GPU; "host" pointers are read or
 *   written synchronously before the call returns.
 * - Calls enqueue on `stream` (a hipStream_t, NULL = the null stream) and
 *   return; results are ready when the stream reaches them.  Only
 *   ttm_find_peaks synchronises (it returns the peak count to the host).
 * - Errors: argument checks are synchronous and return a negative
 *   ttm_status without enqueuing anything; ttm_last_error() gives a message
 *   (per calling thread).  Device faults surface as TTM_EDEVICE from the next
 *   call that observes them.  Nothing aborts or throws across the ABI.
 * - Workspace: entry points taking (ws, ws_bytes) need a device scratch
 *   buffer of at least ttm_workspace_size(...) bytes, 256-byte aligned; they
 *   return TTM_EWORKSPACE if it is smaller.  They allocate nothing.
 * - Thread safety: one context per host thread; calls that share a workspace
 *   must be ordered on one stream.
 */
#ifndef TTM_H_
#define TTM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TTM_OK = 0,
  TTM_EINVAL = -1,        /* bad argument (shape, degree, pointer, option) */
  TTM_ENOMEM = -2,        /* context allocation failed                      */
  TTM_EDEVICE = -3,       /* HIP runtime or device error                    */
  TTM_EUNSUPPORTED = -4,  /* valid request outside what the library computes */
  TTM_EWORKSPACE = -5     /* workspace smaller than ttm_workspace_size()    */
} ttm_status;

typedef enum { TTM_F32 = 0, TTM_BF16 = 1 } ttm_dtype;

/* Operations for ttm_workspace_size. */
typedef enum {
  TTM_OP_SPECTRA = 1,
  TTM_OP_NORMALIZE = 2,
  TTM_OP_CORRELATE = 3,
  TTM_OP_PEAKS = 4,
  TTM_OP_EXTRACT = 5,     /* nz x ny x nx = the extraction box            */
  TTM_OP_MLP_TRAIN = 6,   /* nz = batch size, ny = nx = 1                 */
  TTM_OP_PREFILTER = 7,   /* nz x ny x nx = the volume (fft_n unused)     */
  TTM_OP_REFINE = 8,      /* nz = peaks, ny = the refinement radius r_s
                             rounded up (the size covers every smaller r_s) */
  TTM_OP_TENSOR_WEDGE = 9, /* ttm_build_tensor_wedge (fft_n, nz, ny, nx unused) */
  TTM_OP_NORM_CORR = 10    /* ttm_normalize_correlate (nz, ny, nx unused) */
} ttm_op;

typedef struct ttm_ctx ttm_ctx;

/* Geometry and method constants. */
typedef struct {
  int32_t degree;       /* n, even, 0..8                                    */
  int32_t dprime;       /* 3 (template-axis form) or 4 (quaternion form)    */
  int32_t L;            /* template edge, 2..64                             */
  float mask_radius;    /* r, 0 < r < L/2                                   */
  float filter_a;       /* a of the filter 1 + a(z + 1/z - 2), 0 < a < 1/4  */
  float eps_w;          /* w = 0 where var <= eps_w * M * mean(g^2)         */
  float axis[3];        /* d' = 3: template axis a (unit), default (0,0,1)  */
} ttm_desc;

/* Context: owns the per-device FFT twiddle tables. */
int ttm_create(ttm_ctx** out, int device);
void ttm_destroy(ttm_ctx* ctx);
const char* ttm_last_error(void);

/* K = binom(n + d' - 1, n), or -1 for an unsupported (n, d'). */
int ttm_n_components(int degree, int dprime);
/* Complex (float2) elements of one half spectrum of an N^3 real array:
 * N * (N/2 + 1) * N.  Spectra are stored [kz][kx][ky] (ky fastest). */
size_t ttm_spectrum_elems(int fft_n);
/* Complex elements of one template spectrum from ttm_template_spectra:
 * L * (N/2 + 1) * N, or 0 for an unsupported edge or L outside 1..fft_n. */
size_t ttm_template_spectrum_elems(int fft_n, int L);
/* FFT edges the library supports (32, 64, 128, 256, 512 and the mixed-radix
 * 96, 160, 192): 1 if supported. */
int ttm_fft_supported(int fft_n);

/* Workspace bytes for an operation at FFT edge fft_n on an nz x ny x nx
 * volume (0 for an invalid request). */
size_t ttm_workspace_size(const ttm_desc* desc, int op, int fft_n, int nz, int ny, int nx);

/*
 * Tensor template, Eq. tt and Alg. 1 (one-time per template).
 *   t'    = m (S(t) - mu) / sigma_t        (Eq. norm_t; S(t) = m (h * t), zero padding)
 *   T_a(p) = (1/nq) sum_q v_q^a t'(c + R(q)^T (p - c))
 * with trilinear interpolation, zero outside the box, and v_q = R(q) axis
 * (d' = 3) or v_q = q (d' = 4).
 *   tmpl   device, L^3 float
 *   quats  device, nq x 4 float unit quaternions (w, x, y, z), equal weights
 *   T_out  device, K x L^3 float
 *   tn_out device, L^3 float: receives t' (required; also the working copy)
 * Errors: TTM_EINVAL for nq < 1, null pointers, bad desc.
 */
int ttm_build_tensor(ttm_ctx* ctx, const ttm_desc* desc, const float* tmpl,
                     const float* quats, int nq, float* T_out, float* tn_out, void* stream);

/*
 * Wedge-aware tensor template (a reading of Eq. tt for tomograms with a
 * missing wedge; the paper does not treat the wedge).  As ttm_build_tensor,
 * but every rotated template passes through the tomogram's missing-wedge
 * filter and is renormalised over the mask before it is added:
 *   T_a(p) = (1/nq) sum_q v_q^a N_m(W t'_q)(p)
 * t'_q = t' rotated by R(q) (trilinear, as ttm_build_tensor); W zeroes the
 * Fourier coefficients with |k_z| > tan(wedge_deg) |k_x| (tilt axis y, beam z;
 * DC kept), applied on the template box zero-padded to P^3, P the smallest
 * power of two >= max(L, 32) (periodic transform); N_m(v) = m (v - mu) / sigma
 * with mu = <v, m>/M and sigma^2 = <v^2, m> - <v, m>^2/M (Eq. norm_t without
 * a second prefilter).  The wedge lies in the tomogram's frame, so it acts
 * after each rotation: filtering t' once before Alg. 1 would turn it with the
 * template.  Correlating a wedged tomogram with T then scores every rotation
 * by the part of the template the tomogram can show.
 *   wedge_deg  half-angle in (0, 90) degrees (60 for a +-60 degree tilt range)
 *   ws         ttm_workspace_size(desc, TTM_OP_TENSOR_WEDGE, 0, 0, 0, 0) bytes
 * Other arguments as ttm_build_tensor.  Errors: TTM_EINVAL as there, or for
 * wedge_deg outside (0, 90); TTM_EUNSUPPORTED for L > 512; TTM_EWORKSPACE.
 */
int ttm_build_tensor_wedge(ttm_ctx* ctx, const ttm_desc* desc, const float* tmpl,
                           const float* quats, int nq, float wedge_deg, float* T_out,
                           float* tn_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Spectra of the template fields for correlation at FFT edge fft_n (Alg. 2,
 * F(T_i)): each field is placed at the origin of a zero N^3 array and
 * forward-transformed (unnormalised e^{-i}) along x and y.  Only z planes
 * 0..L-1 of such an array are nonzero, and only those are stored: the z
 * transform is taken inside ttm_correlate / ttm_normalize, column by column,
 * so each tile reads L/N of the bytes of full spectra.  Output: K component
 * arrays followed by the one of the mask m, (K + 1) x
 * ttm_template_spectrum_elems(N, L) float2, device, each [z < L][kx][ky]
 * (ky fastest, kx in 0..N/2).  Requires L <= fft_n.
 */
int ttm_template_spectra(ttm_ctx* ctx, const ttm_desc* desc, const float* T, int fft_n,
                         void* spec_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Prefilter and local normalisation (Sec. 2, Eq. norm_f).
 *   g_out = h * vol (3-tap separable, border voxels replicated), full size
 *   w_out(x) = 1/sqrt(var(x)) on the valid region, 0 elsewhere, where
 *     var(x) = sum_p m(p) g(x+p-c)^2 - (sum_p m(p) g(x+p-c))^2 / M
 *   evaluated by FFT correlation with the mask on fft_n^3 tiles, with the
 *   data centred by the volume mean and the difference formed in FP64;
 *   w = 0 where var <= eps_w * M * mean(g^2).
 *   stats_out device double[2]: {mean(g), mean(g^2)} over the volume.
 *   mask_spec: the mask spectrum from ttm_template_spectra at fft_n.
 */
int ttm_normalize(ttm_ctx* ctx, const ttm_desc* desc, const float* vol, int nz, int ny,
                  int nx, const void* mask_spec, int fft_n, float* g_out, float* w_out,
                  double* stats_out, void* ws, size_t ws_bytes, void* stream);

/*
 * The two halves of ttm_normalize, so that the local normalisation of one
 * tile can run just before that tile's correlation (Sec. 2, Eq. norm_f).
 * ttm_prefilter: g_out = h * vol and stats_out = {mean(g), mean(g^2)} as in
 *   ttm_normalize; if w_out is not NULL it is cleared to 0 (the value outside
 *   the valid region).  ws: ttm_workspace_size(desc, TTM_OP_PREFILTER, 0, nz,
 *   ny, nx) bytes.
 * ttm_normalize_box: w_out on the box (host int32[3] lo and size, z y x,
 *   inside the valid region) from g and stats of ttm_prefilter, computed on
 *   the same fft_n^3 sub-tiles as ttm_normalize, so a partition of the valid
 *   region into boxes aligned to the step fft_n - L + 1 from the valid corner
 *   reproduces ttm_normalize's w bit for bit.  ws: ttm_workspace_size(desc,
 *   TTM_OP_NORMALIZE, fft_n, nz, ny, nx) bytes.
 */
int ttm_prefilter(ttm_ctx* ctx, const ttm_desc* desc, const float* vol, int nz, int ny, int nx,
                  float* g_out, float* w_out, double* stats_out, void* ws, size_t ws_bytes,
                  void* stream);
int ttm_normalize_box(ttm_ctx* ctx, const ttm_desc* desc, const float* g, int nz, int ny, int nx,
                      const double* stats, const void* mask_spec, int fft_n,
                      const int32_t box_lo[3], const int32_t box_size[3], float* w_out, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * Tensor field on a box of the valid region (Eq. tcc, Alg. 2):
 *   C_a(x) = w(x) * F^{-1}{ F(g) conj(F(T_a)) }(x)   for x in the box
 * computed on fft_n^3 tiles (each tile yields (fft_n - L + 1)^3 outputs).
 *   g, w     device, nz x ny x nx float (from ttm_normalize)
 *   stats    device double[2] from ttm_normalize (the mean centres the FFT input)
 *   spec     device, component spectra from ttm_template_spectra at fft_n
 *   box_lo   host int32[3] (z, y, x) first voxel; box_size host int32[3];
 *            the box must lie in the valid region
 *   C_out    device, K x bz x by x bx, float32 or bfloat16 (out_dtype)
 */
int ttm_correlate(ttm_ctx* ctx, const ttm_desc* desc, const float* g, const float* w,
                  int nz, int ny, int nx, const double* stats, const void* spec, int fft_n,
                  const int32_t box_lo[3], const int32_t box_size[3], int out_dtype,
                  void* C_out, void* ws, size_t ws_bytes, void* stream);

/*
 * ttm_normalize_box followed by ttm_correlate on one FFT tile, sharing the
 * tile's forward transform of the centred g (both calls transform the same
 * tile of g; the results equal those of the two calls, bit for bit):
 *   w_out on the box (Eq. norm_f), then C_out = w * F^{-1}{F(g) conj(F(T_a))}.
 *   spec       the template planes from ttm_template_spectra; their last
 *              entry (index K) is the mask's, as for ttm_normalize_box
 *   box_lo, box_size  host int32[3]: inside the valid region, at most
 *              fft_n - L + 1 voxels along each axis (one tile)
 *   ws         ttm_workspace_size(desc, TTM_OP_NORM_CORR, fft_n, 0, 0, 0) bytes
 * Other arguments as the two calls.  Errors: as theirs, and TTM_EINVAL for a
 * box larger than one tile.
 */
int ttm_normalize_correlate(ttm_ctx* ctx, const ttm_desc* desc, const float* g, int nz, int ny,
                            int nx, const double* stats, const void* spec, int fft_n,
                            const int32_t box_lo[3], const int32_t box_size[3], float* w_out,
                            int out_dtype, void* C_out, void* ws, size_t ws_bytes, void* stream);

/* ttm_extract mode bits. */
#define TTM_SCORE 1       /* write c = ||C||_F                                   */
#define TTM_ORIENT 2      /* write lambda and u (dominant eigenpair by SS-HOPM)  */
#define TTM_START_MLP 4   /* seed SS-HOPM from the MLP; fall back to multistart  */
#define TTM_START_ONLY 8  /* with TTM_START_MLP: write the network's unit start
                             direction to dir (lambda = 0), no search          */
#define TTM_NO_SCREEN 16  /* with TTM_START_MLP: skip the fixed-start screening
                             (fall back only on kappa or non-convergence)      */

typedef struct {
  int32_t mode;            /* TTM_SCORE | TTM_ORIENT [| TTM_START_MLP]            */
  int32_t n_starts;        /* number of fixed start vectors, 1..64                */
  const float* starts;     /* device, n_starts x d' unit vectors                  */
  const void* mlp;         /* device, packed MLP parameters (ttm_mlp_pack), or NULL */
  float fallback_kappa;    /* learned start: fall back when lambda < kappa * c, or
                              when SS-HOPM from the learned start did not reach tol */
  int32_t max_iter;        /* SS-HOPM update cap per start, 1..2^24               */
  float tol;               /* stop when |delta lambda| <= tol (on C / ||C||_F)    */
  int32_t newton_steps;    /* Newton polishing steps per answer, 0..8 (default 2) */
  uint64_t* work_counters; /* device uint64[5] or NULL: adds {SS-HOPM updates,
                              Newton steps, oriented voxels, shift bounds computed,
                              SS-HOPM runs started} of this call (for FLOP counts;
                              counting costs atomics per wavefront, so leave it
                              NULL where the call is timed) */
} ttm_extract_opts;

/*
 * Per-voxel score and orientation (Sec. 3.1, 3.2) for a box of field values.
 *   C         device, K x bz x by x bx (in_dtype float32 or bfloat16)
 *   score     device map or NULL; lambda device map or NULL; dir device map
 *             (d' floats per voxel, [z][y][x][d']) or NULL
 *   out_lo    host int32[3]: where voxel (0,0,0) of the box lands in the maps
 *   out_dims  host int32[3]: extent (z, y, x) of the output maps
 *   n_fallback device int32 counter incremented per voxel whose learned start
 *             fell back to the multistart search, or NULL
 *   ws        device workspace of ttm_workspace_size(desc, TTM_OP_EXTRACT, 0,
 *             bz, by, bx) bytes (run queues, per-run results and the tensors
 *             the learned start hands on, about 430 bytes per box voxel at
 *             degree 6); required with TTM_ORIENT, may be NULL for
 *             TTM_SCORE alone.  Calls that share a workspace must be ordered
 *             on one stream.
 * Orientation: alpha = max(0, -lambda_min(U)) with U the square unfolding of
 * C/||C||_F (lambda_min of the unfolding's symmetric block bounded from below:
 * its Gershgorin interval narrowed by 12 bisection steps with Cholesky tests,
 * minus 1e-5, so alpha is never below the rule's value); SS-HOPM u <- (C u^{n-1} + alpha u)/||.|| from every start
 * until |delta lambda| <= tol or max_iter updates, then up to newton_steps
 * Riemannian Newton steps (taken where the tangent Hessian
 * (n-1) E^T (C u^{n-2}) E - lambda I is negative definite, kept unless lambda
 * drops by more than 1e-7); the largest lambda wins (first on ties); u is
 * signed so its last non-zero coordinate is positive (d' = 3) or its w is
 * (d' = 4).  The (voxel, start) runs are spread over the GPU's lanes from a
 * work queue, so a slow run does not hold up other voxels.
 * Learned start (TTM_START_MLP): per wavefront of 64 voxels the network
 * (ttm_mlp_train_step) maps x = sqrt(mu_a) C_a / ||C||_F to a start direction
 * on the BF16 matrix cores.  d' = 3: up to five guarded Newton steps from it,
 * else SS-HOPM from it and the Newton polish; d' = 4: SS-HOPM from it and the
 * Newton polish.  The end point must then be certified near a local maximum
 * (tangent gradient <= 3e-5 with no tangent-Hessian eigenvalue above 1e-3, or
 * a negative definite tangent Hessian and a Newton step <= 0.01, after up to
 * four more guarded Newton steps).  Voxels whose result is not converged, not
 * certified, has lambda < fallback_kappa * ||C||_F, or is beaten by the value
 * of <C, s^n> at one of the fixed starts s (SS-HOPM never lowers lambda, so
 * the multistart answer is then higher) are queued for the multistart search
 * above; the better of the two answers is kept.  Requires lambda and dir.
 */
int ttm_extract(ttm_ctx* ctx, const ttm_desc* desc, const void* C, int in_dtype,
                const int32_t box_size[3], const ttm_extract_opts* opts, float* score,
                float* lambda, float* dir, const int32_t out_lo[3], const int32_t out_dims[3],
                int32_t* n_fallback, void* ws, size_t ws_bytes, void* stream);

/*
 * ttm_extract without a workspace argument, for callers that cannot allocate
 * device memory (code under stream / graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, rules and results as
 * ttm_extract; the scratch is a 64 MiB array the library holds on each GPU
 * it runs on (about 150 000 box voxels at degree 6), so the call allocates
 * nothing.  A box whose orientation scratch would exceed it is rejected with
 * TTM_EUNSUPPORTED before anything is enqueued.  Every call on one GPU shares
 * that array (the kernels clear what must start at zero): calls that overlap
 * on one GPU, on any streams, race and must be ordered by the caller.
 */
int ttm_extract_noalloc(ttm_ctx* ctx, const ttm_desc* desc, const void* C, int in_dtype,
                        const int32_t box_size[3], const ttm_extract_opts* opts, float* score,
                        float* lambda, float* dir, const int32_t out_lo[3],
                        const int32_t out_dims[3], int32_t* n_fallback, void* stream);

/*
 * Position refinement TTM-ref (Sec. 3.3, Alg. 3), quaternion form (d' = 4,
 * degree 2, 4 or 6).  For each peak x^i (device int32 n_peaks x 3, z y x, inside
 * the valid region, e.g. from ttm_find_peaks) the voxels of the sphere
 * |x - x^i| <= r_s are visited, the peak first and then the other offsets in
 * lexicographic (dz, dy, dx) order; voxels whose template window leaves the
 * volume are skipped.  At each voxel x:
 *   C(x)    = w(x) sum_p g(x + p - c) T_a(p)        (Eq. tcc, real-space sums)
 *   R(x)    = the optimal rotation of C(x): the multistart SS-HOPM of
 *             ttm_extract on S^3 (opts: n_starts quaternion starts, max_iter,
 *             tol, newton_steps; mode, mlp and kappa are ignored)
 *   c(x)    = w(x) sum_p g(x + p - c) t'(c + R(x)^T (p - c))  (Eq. lncc at R(x))
 * and the voxel of the largest c is kept (a later voxel only on a strictly
 * larger value, so the peak stays on ties).  Reading of the printed
 * algorithm: its loop runs over the sphere of x^i, and the search starts at
 * x^i with the peak's own rotation and LNCC.
 *   g, w      device, nz x ny x nx (from ttm_prefilter / ttm_normalize_box)
 *   T         device, K x L^3 tensor template (ttm_build_tensor, d' = 4)
 *   tn        device, L^3 normalised template t' (ttm_build_tensor's tn_out)
 *   r_s       0 <= r_s < 9 (the paper uses 3)
 *   pos_out   device int32 n_peaks x 3: refined positions (z, y, x)
 *   quat_out  device float n_peaks x 4: their rotations (w, x, y, z), w >= 0
 *   lncc_out  device float n_peaks: their LNCC
 *   quat_peak_out, lncc_peak_out  device, optional (NULL): the rotation and
 *             LNCC at each unrefined peak (TTM without refinement)
 *   ws        ttm_workspace_size(desc, TTM_OP_REFINE, 0, n_peaks, ceil(r_s), 1) bytes
 * Errors: TTM_EUNSUPPORTED unless d' = 4 and degree 2, 4 or 6; TTM_EINVAL for
 * null pointers, n_peaks < 1 or r_s out of range.
 */
int ttm_refine(ttm_ctx* ctx, const ttm_desc* desc, const float* g, const float* w, int nz, int ny,
               int nx, const float* T, const float* tn, const int32_t* peaks, int n_peaks, float r_s,
               const ttm_extract_opts* opts, int32_t* pos_out, float* quat_out, float* lncc_out,
               float* quat_peak_out, float* lncc_peak_out, void* ws, size_t ws_bytes,
               void* stream);

/*
 * ttm_extract over many boxes in one call (d' = 3 or 4): a batch of subtomograms
 * whose field boxes share the descriptor (and, with TTM_START_MLP, the
 * network), extracted by the same launches as one box of total_voxels
 * voxels, so a batch costs about the kernels of one call instead of one call
 * per box.  Rules, options and results per voxel are those of ttm_extract.
 *   items       device array of n_items ttm_extract_item; item i's voxels are
 *               numbers first_i .. first_i + its box volume - 1 of the batch,
 *               with first_0 = 0 and first_{i+1} = first_i + box volume of i
 *               (the caller's responsibility, as are the pointers: field
 *               planes K x box, maps of out_dims holding the box at out_lo;
 *               score may be NULL without TTM_SCORE; lambda and dir are
 *               required with TTM_ORIENT)
 *   total_voxels the batch's voxel count (sum of the box volumes)
 *   ws          ttm_workspace_size(desc, TTM_OP_EXTRACT, 0, total_voxels, 1, 1) bytes
 * Errors: as ttm_extract (the same degree and learned-start limits per form).
 */
typedef struct {
  const void* C;            /* device, K x box[0] x box[1] x box[2] (in_dtype)  */
  float* score;             /* device map or NULL                               */
  float* lambda;            /* device map or NULL                               */
  float* dir;               /* device map (d' floats per voxel) or NULL         */
  uint64_t first;           /* index of the box's first voxel in the batch      */
  int32_t box[3];           /* bz, by, bx                                       */
  int32_t out_lo[3];        /* where box voxel (0,0,0) lands in the maps        */
  int32_t out_dims[3];      /* extent (z, y, x) of the maps                     */
  int32_t reserved;
} ttm_extract_item;

int ttm_extract_batch(ttm_ctx* ctx, const ttm_desc* desc, const ttm_extract_item* items,
                      int n_items, uint64_t total_voxels, int in_dtype,
                      const ttm_extract_opts* opts, int32_t* n_fallback, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * Learned start network (a seed for the orientation search of Sec. 3.1), for
 * d' = 3 at degree 2, 4, 6 and d' = 4 at degree 2, 4:
 * x (K features, zero padded to kin = 32 when K <= 32, else 48) -> 64 -> relu
 * -> 64 -> relu -> d', BF16 weights, FP32 accumulation, activations rounded
 * to BF16.  FP32 master parameters (ttm_mlp_param_count(desc) floats, layout
 * W1[kin][64], b1[64], W2[64][64], b2[64], W3[64][16], b3[16]; rows of W1
 * beyond K and columns of W3 beyond d' are kept 0); packed inference copy of
 * ttm_mlp_packed_bytes(desc) bytes.  Both return 0 for a form or degree
 * without a learned start.
 */
size_t ttm_mlp_param_count(const ttm_desc* desc);
size_t ttm_mlp_packed_bytes(const ttm_desc* desc);
/* packed = BF16 fragment-ordered copy of params (device -> device), for the
 * network of desc's form and degree. */
int ttm_mlp_pack(ttm_ctx* ctx, const ttm_desc* desc, const float* params, void* packed,
                 void* stream);
/*
 * One training step on B pairs: C device B x K raw tensors (row per sample),
 * targets device B x d' directions (axes, or quaternions at d' = 4).  Loss mean(1 - (u.t/|t|)^2), u =
 * y/|y| (sign invariant).  Adam (beta 0.9, 0.999, eps 1e-8, bias corrected,
 * step >= 1) on params with moments adam_m, adam_v (device, param_count
 * floats each) when lr > 0.  Optional outputs: packed (updated inference
 * copy), loss_out (device float, loss before the update), grads_out (device,
 * param_count floats).  ws: ttm_workspace_size(desc, TTM_OP_MLP_TRAIN, 0, B, 1, 1).
 */
int ttm_mlp_train_step(ttm_ctx* ctx, const ttm_desc* desc, const float* C, const float* targets,
                       int B, float* params, float* adam_m, float* adam_v, int step, float lr,
                       void* packed, float* loss_out, float* grads_out, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Find Peaks (Sec. 3.4): visit the voxels of [valid_lo, valid_hi] (inclusive,
 * z y x) in descending score, ties by ascending linear index z*ny*nx + y*nx + x,
 * and keep a voxel when its Euclidean distance to every kept peak is
 * >= min_dist; stop after top_p peaks.
 *   peaks_out device int32 top_p x 3 (z, y, x); vals_out device float top_p
 *   n_found   host int32: number of peaks written (synchronises the stream)
 */
int ttm_find_peaks(ttm_ctx* ctx, const float* score, int nz, int ny, int nx,
                   const int32_t valid_lo[3], const int32_t valid_hi[3], int top_p,
                   float min_dist, int32_t* peaks_out, float* vals_out, int32_t* n_found,
                   void* ws, size_t ws_bytes, void* stream);

/*
 * Find Peaks with the same rule and result as ttm_find_peaks, for callers
 * that cannot synchronise (e.g. under stream / graph capture): every valid
 * voxel is a candidate (sorted on the device), nothing is copied to the host,
 * and the number of peaks found is written to the device int32 n_found.
 * Workspace as ttm_find_peaks; the volume must hold fewer than 2^31 voxels.
 */
int ttm_find_peaks_async(ttm_ctx* ctx, const float* score, int nz, int ny, int nx,
                         const int32_t valid_lo[3], const int32_t valid_hi[3], int top_p,
                         float min_dist, int32_t* peaks_out, float* vals_out, int32_t* n_found,
                         void* ws, size_t ws_bytes, void* stream);

/*
 * Find Peaks over many score maps in one launch (Sec. 3.4, the rule and
 * result of ttm_find_peaks for each map), for batches of subtomograms that
 * each want a few peaks.  Each step keeps the first voxel in visiting order
 * (descending score, ties by ascending linear index) at least min_dist from
 * the peaks kept so far, i.e. the smallest key ~score_bits << 32 | index
 * among the voxels not yet excluded; no host synchronisation (graph-capture
 * safe).  Work per map is about top_p times the voxels of an exclusion ball,
 * so it suits small top_p (ttm_find_peaks serves thousands of peaks better).
 *   items     device array of n_items ttm_peak_item (the table itself lives
 *             on the device so a captured graph can replay it)
 *   max_valid host int32[3]: the largest valid-box extent (z, y, x) of any item
 * Per item (the caller's responsibility; an item that breaks these gets
 * *n_found = -1 and is skipped): valid box inside the map, map under 2^32
 * voxels, 1 <= top_p <= 4096, scratch of ttm_peaks_batch_scratch_bytes(
 * valid_lo, valid_hi) bytes (256-byte aligned, overwritten).
 */
typedef struct {
  const float* score;       /* device map, dims[0] x dims[1] x dims[2]          */
  int32_t* peaks;           /* device int32 top_p x 3 (z, y, x)                 */
  float* vals;              /* device float top_p: the scores of the peaks      */
  int32_t* n_found;         /* device int32: the number of peaks written        */
  void* scratch;            /* device scratch of this item                      */
  int32_t dims[3];
  int32_t valid_lo[3];      /* inclusive valid box (z, y, x)                    */
  int32_t valid_hi[3];
  int32_t top_p;
  float min_dist;
} ttm_peak_item;

size_t ttm_peaks_batch_scratch_bytes(const int32_t valid_lo[3], const int32_t valid_hi[3]);
int ttm_find_peaks_batch(ttm_ctx* ctx, const ttm_peak_item* items, int n_items,
                         const int32_t max_valid[3], void* stream);

/* Stand-alone 3D FFT of an N^3 real array to its half spectrum and back
 * (the transforms used inside ttm_correlate), for tests and benchmarks.
 * Forward: spec = F(x) unnormalised; inverse: x = F^{-1}(spec) * scale.
 * The inverse overwrites spec. */
int ttm_fft3d_r2c(ttm_ctx* ctx, const float* x, int fft_n, void* spec, void* stream);
int ttm_fft3d_c2r(ttm_ctx* ctx, void* spec, int fft_n, float scale, float* x, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TTM_H_ */
