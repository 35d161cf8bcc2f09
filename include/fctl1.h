/*
 * fctl1 -- Fast Cauchy Transform l1 regression on AMD MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of FastCauchyRegression (Clarkson,
 * Drineas, Magdon-Ismail, Mahoney, Meng, Woodruff, "The Fast Cauchy Transform
 * and Faster Robust Linear Regression", arXiv 1207.4684):
 *
 *   fct_sketch       Pi1 X with the FCT1 transform Pi1 = 4 B C H~
 *                    (Section "FCT1 Construction"), optional FP64 R of its QR
 *                    (figure FastL1Basis; regression figure steps 1-2);
 *   l1_sample_probs  lambda_i = median_j |(X R^-1 Pi2)_ij| and
 *                    p_i = min{1, s lambda_i / sum lambda} (steps 3-6);
 *   l1_coreset       steps 1-7: the kept rows, their weights 1/p_i and the
 *                    gathered coreset (D A, D b) without the weights applied;
 *   l1_regress       steps 1-8: x_hat = argmin ||D A x - D b||_1 (step 8 by
 *                    FP64 iteratively reweighted least squares on the GPU).
 *   fct2_sketch      Pi1 X with the FCT2 transform (Section "FCT2
 *                    Construction"), optional R; FCT_FLAG_FCT2 makes
 *                    l1_regress take its R from it.
 *
 * Conventions shared by every entry point:
 *   - X = [A, -b] has n rows and q = d + 1 columns when b != NULL, else X = A
 *     and q = d.  A is column-major: element (i, j) at A[i + j * lda], lda >= n.
 *     b is a length-n vector of the same type.  All array arguments are DEVICE
 *     pointers unless marked "host"; the caller owns every buffer it passes.
 *   - The library owns only the scratch memory inside its context.
 *   - Every call is enqueued on the context's HIP stream; a call with host
 *     outputs waits for the stream before it returns.
 *   - Arguments are checked before anything is launched; on an error no output
 *     is written.  Status codes are the FCT_* values below (0 = success); no
 *     C++ exception crosses the interface.
 *   - Random quantities come from Philox4x32-10 with key = seed and counters
 *     (index, 0, stream, 0) as listed in the design notes; the same seed gives
 *     the same Pi1, Pi2 and sampling decisions as the CPU oracle.
 *   - Sketch sums of FP32 data with s <= 1024 and r1 <= 1024 are formed by one
 *     lane each in an order fixed by the random streams, so repeated calls
 *     give bitwise-identical Y, R, lambda, probabilities, coresets and
 *     solutions.  Other shapes add into LDS atomically (FP64 data, s > 1024,
 *     r1 > 1024) and repeated runs agree to rounding, unless the call sets
 *     FCT_FLAG_DETERMINISTIC (FP32 data with s <= 1024; at r1 > 1024 the
 *     buckets are split over ceil(r1 / 1024) workgroups, each streaming X
 *     again).  Integer and index outputs (RNG words, buckets, signs, selected
 *     rows given the same probabilities) are exact.
 */
#ifndef FCTL1_H
#define FCTL1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fct_ctx fct_ctx;

typedef enum { FCT_F32 = 0, FCT_F64 = 1, FCT_BF16 = 2 } fct_dtype;

enum {
  FCT_OK = 0,
  FCT_ERR_BAD_ARG = -1,        /* an argument is out of range or NULL         */
  FCT_ERR_OOM = -2,            /* device scratch could not be allocated        */
  FCT_ERR_NONFINITE = -3,      /* NaN or Inf met in an input                   */
  FCT_ERR_RANK_DEFICIENT = -4, /* |R_jj| <= tol ||R[:, j]||_2 (tol 1e-13 for FP64 input,
                                  1e-5 for FP32), or a singular coreset system
                                  (the solver's first, unreweighted system)    */
  FCT_ERR_HIP = -5,            /* a HIP runtime call failed                    */
  FCT_ERR_CAPACITY = -6        /* realised coreset size exceeds the capacity   */
};

/* Flags of fct_params.flags and of fct_sketch. */
#define FCT_FLAG_NO_SIGN_FLIP 1u /* Pi1 without the random sign diagonal: the paper's Pi1 exactly */
#define FCT_FLAG_GAUSSIAN_PI2 4u /* optimized regression: Pi2 of standard Gaussians (figure
                                    OptimizedFastCauchyRegression), see l1_sample_probs_ex */
#define FCT_FLAG_FCT2 8u /* l1_regress / l1_coreset: R from the FCT2 sketch (fct2_sketch with
                             t = s, s = s2) instead of FCT1; other entry points reject it */
#define FCT_FLAG_DETERMINISTIC 2u /* bitwise-reproducible sketch at any r1 (FP32 data, s <= 1024;
                                     FCT_ERR_BAD_ARG for other shapes)                        */

typedef struct {
  int32_t s;      /* FWHT block size: power of two in [2, 4096]                  */
  int32_t r1;     /* rows of Pi1 (sketch rows), q <= r1 <= 65536                 */
  int32_t r2;     /* columns of Pi2, 1 <= r2 <= 32                               */
  int32_t s2;     /* FCT_FLAG_FCT2 only: rows G keeps per block of s, 1 <= s2 <= min(s, 256) */
  int64_t s_out;  /* expected coreset size: the paper's s in step 6 (> 0)        */
  uint64_t seed;  /* key of every random stream                                  */
  uint32_t flags; /* FCT_FLAG_*                                                   */
  int32_t irls_iters; /* step 8 iteration cap (<= 0: library default)            */
} fct_params;

/* Context: binds a device and a HIP stream (hip_stream == NULL: the library
 * creates its own stream).  *ctx receives the handle.  Status code. */
int fct_create(fct_ctx **ctx, int device, void *hip_stream);
/* Frees the context's scratch and stream (if it created it). NULL is a no-op. */
void fct_destroy(fct_ctx *ctx);
/* Static text for a status code. */
const char *fct_strerror(int status);
/* Waits for all work queued on the context's stream and returns (then clears)
 * the first condition the device flagged since the last wait:
 * FCT_ERR_NONFINITE or FCT_ERR_RANK_DEFICIENT; FCT_OK otherwise. */
int fct_sync(fct_ctx *ctx);
/* The HIP stream the context enqueues on (hipStream_t as void*). */
void *fct_stream(fct_ctx *ctx);

/*
 * fct_sketch: Y = Pi1 X (FCT1 section; regression figure step 2).
 *   A, lda, b  as above; dt = FCT_F32 or FCT_F64 (A and b of that type).
 *   n >= 1, 1 <= d, q <= r1; s a power of two in [2, 4096]; rows are padded
 *   with zeros to s * ceil(n / s).
 *   Y: device, r1 x q column-major (ld = r1), of type dt.  May be NULL when
 *      only R is wanted.
 *   R: device, q x q column-major FP64, upper triangular with positive
 *      diagonal, Pi1 X = Q R (may be NULL).  Requires q <= 88.
 *   flags: FCT_FLAG_NO_SIGN_FLIP, FCT_FLAG_DETERMINISTIC (see above) or 0.
 *   Conditions found on the device (a non-finite input, a rank-deficient
 *   sketch) are reported by the next fct_sync on the context (the call
 *   itself does not wait): FCT_ERR_NONFINITE, FCT_ERR_RANK_DEFICIENT.
 */
int fct_sketch(fct_ctx *ctx, const void *A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
               const void *b, int32_t s, int32_t r1, uint64_t seed, uint32_t flags,
               void *Y, double *R);

/*
 * fct_sketch_window: the share of Pi1 X contributed by rows
 * [row0, row0 + n) of a larger design.  Pi1 acts block by block (FCT1
 * section: H~ is block diagonal, and B and C act on stacked positions), so
 * with every random stream indexed by the global row the sketches of
 * consecutive windows add up to the sketch of their union.  This is how a
 * design split across devices or streamed in pieces is sketched.
 *   A, b: device pointers to the window's first row (element (row0 + i, j)
 *         of the whole design at A[i + j * lda]); n rows in the window.
 *   row0: global index of the window's first row; a multiple of s and of
 *         256, else FCT_ERR_BAD_ARG.  The last window may end anywhere: rows
 *         past its end count as zero padding of the whole design.
 *   Other arguments and Y as in fct_sketch (no R: a window has no basis).
 */
int fct_sketch_window(fct_ctx *ctx, const void *A, int64_t n, int32_t d, int64_t lda,
                      fct_dtype dt, const void *b, int32_t s, int32_t r1, uint64_t seed,
                      int64_t row0, uint32_t flags, void *Y);

/*
 * fct2_sketch: Y = Pi1 X with the FCT2 transform (section "FCT2
 * Construction", Theorem FCT2): Pi1 = 8/r1 sqrt(pi t / (2 s)) C Hbar, Hbar
 * block-diagonal with ceil(n / t) copies of the s x t matrix
 * G = sqrt(t/s) P H_t D, C an r1 x (ceil(n / t) s) matrix of independent
 * standard Cauchy variates.  The paper only asks G to be a fast
 * Johnson-Lindenstrauss transform; here G is the subsampled randomized
 * Hadamard transform: D random signs (the stream FCT1 uses), H_t the
 * normalized Hadamard matrix of order t, P keeping s of the t rows drawn
 * uniformly with replacement.  Rows are padded with zeros to
 * t * ceil(n / t).  Every random entry comes from the seed (Philox streams
 * 1, 5 and 6), so the call is deterministic and bitwise reproducible.
 *   A, lda, b, dt  as in fct_sketch (FCT_F32 or FCT_F64; X = [A, -b] when b
 *         is not NULL, q = d + 1; X = A otherwise, q = d).
 *   t: power of two in [64, 4096]; s: 1 <= s <= min(t, 256); q <= r1 <= 65536.
 *   Y: device, r1 x q column-major (ld = r1), of type dt, or NULL.
 *   R: device, q x q column-major FP64 upper triangular, Pi1 X = Q R, or
 *      NULL (q <= 88).  Y and R may not both be NULL.
 *   Scratch: (ceil(n/t) s) x q FP64 for G applied to every block, plus
 *   partial sums of about 4096 / ceil(r1 / 256) chunks of r1 x q FP64.
 *   Device conditions as in fct_sketch.
 */
int fct2_sketch(fct_ctx *ctx, const void *A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
                const void *b, int32_t t, int32_t s, int32_t r1, uint64_t seed, void *Y,
                double *R);

/*
 * l1_sample_probs: steps 3-6 of the regression figure.
 *   M = R^-1 Pi2 (q x r2, Pi2 of independent Cauchys from the seed) is formed
 *   on the device in FP64, then X is streamed once:
 *   lambda_i = median_j |(X M)_ij| (median of an even count = mean of the two
 *   middle values) and sum_lambda = sum_i lambda_i (FP64).
 *   dt = FCT_F32 or FCT_F64: A and b of that type, contraction in that type.
 *   dt = FCT_BF16: A and b are BF16 copies (same layout); the contraction runs
 *   on bf16 matrix cores with FP32 accumulation and M rounded to BF16.
 *   R: device q x q FP64 from fct_sketch.  1 <= r2 <= 32.  s_out > 0.
 *   lambda: device FP32 [n] or NULL; p: device FP32 [n] (p_i rounded to FP32)
 *   or NULL; sum_lambda: device FP64 scalar or NULL.
 */
int l1_sample_probs(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d,
                    int64_t lda, fct_dtype dt, const double *R, int32_t r2, uint64_t seed,
                    int64_t s_out, float *lambda, float *p, double *sum_lambda);

/*
 * l1_sample_probs_ex: l1_sample_probs with flags.  FCT_FLAG_GAUSSIAN_PI2
 * takes Pi2 of independent standard Gaussians (the optimized regression
 * figure, OptimizedFastCauchyRegression, step 4; Box-Muller from words 0 and 1
 * of stream-2 call a * r2 + c) instead of Cauchys: (U Pi2)_ij is then
 * N(0, ||U_(i)||_2^2) and lambda_i estimates 0.674 ||U_(i)||_2, an l2 row norm
 * within sqrt(q) of the l1 one; fewer columns r2 suffice.  The probabilities
 * are normalized as in the main figure (p_i = min{1, s_out lambda_i / sum
 * lambda}): the optimized figure prints p_i = min{1, s lambda_i} without the
 * sum, while its proof normalizes.  Other flags are ignored.  Other
 * arguments as l1_sample_probs.  fct_params.flags carries the same flag to
 * l1_coreset, l1_regress and l1_regress_batched.
 */
int l1_sample_probs_ex(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d,
                       int64_t lda, fct_dtype dt, const double *R, int32_t r2, uint64_t seed,
                       int64_t s_out, uint32_t flags, float *lambda, float *p,
                       double *sum_lambda);

/*
 * l1_sample_probs_noalloc: l1_sample_probs_ex for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It calls no allocating routine: its
 * scratch (M = R^-1 Pi2 in FP64, FP32 and BF16 forms and the per-workgroup
 * sums of lambda) lives in a static device array of 80 KiB per GPU, held
 * until the process ends.  lambda and sum_lambda must be non-NULL (device
 * FP32 [n] and FP64 scalar); p may be NULL.  q <= 65 (q <= 96 for FCT_F64).
 * FCT_ERR_CAPACITY if the pass-2 grid chosen for n (FCT_OPT_PASS2_WGS) needs
 * more partial sums than the array holds; FCT_ERR_HIP if the array's address
 * could not be found on this device.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two contexts, two host
 * threads) race and must be ordered by the caller.  Nothing in the array has
 * to start at zero (every word a call reads it has written first).  Other
 * arguments and results as l1_sample_probs_ex.
 */
int l1_sample_probs_noalloc(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d,
                            int64_t lda, fct_dtype dt, const double *R, int32_t r2, uint64_t seed,
                            int64_t s_out, uint32_t flags, float *lambda, float *p,
                            double *sum_lambda);

/*
 * l1_coreset: steps 1-7.  Row i is kept iff its stream-3 word is below
 * floor(p_i 2^32) (p_i formed in FP64); kept rows are listed in ascending
 * order.
 *   A, b, dt (FCT_F32 or FCT_F64): the original data, also gathered from.
 *   A_lowp, b_lowp, ld_lowp: optional BF16 copies of A and b streamed by the
 *   sampling pass (NULL: the sampling pass streams A and b).
 *   prm: s, r1, r2, s_out, seed, flags.  cap: capacity in rows of the outputs.
 *   At: device, cap x d column-major (ld = cap), type dt: rows A_idx (unscaled).
 *   bt: device [cap], type dt.  w: device FP64 [cap], 1/p_i.  idx: device
 *   int64 [cap].  S: host, the realised count.  If S > cap the call returns
 *   FCT_ERR_CAPACITY with *S set and the first cap rows written.
 */
int l1_coreset(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d, int64_t lda,
               fct_dtype dt, const void *A_lowp, const void *b_lowp, int64_t ld_lowp,
               const fct_params *prm, int64_t cap, void *At, void *bt, double *w, int64_t *idx,
               int64_t *S);

/*
 * l1_regress: the whole method.  eps documents the acceptance target; when
 * prm->s_out <= 0 the expected coreset size is ceil(20 q / eps).
 *   x: host double[d], the minimizer of the weighted coreset objective (the
 *   iteratively reweighted solve stops at the current iterate when a later,
 *   reweighted system loses a pivot; only a singular first system fails).
 *   obj: host double or NULL, the coreset objective sum_k w_k |A_k x - b_k|.
 *   S_out: host int64 or NULL, the realised coreset size.
 */
int l1_regress(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d, int64_t lda,
               fct_dtype dt, const void *A_lowp, const void *b_lowp, int64_t ld_lowp, double eps,
               const fct_params *prm, double *x, double *obj, int64_t *S_out);

/*
 * One instance of a batch: the arguments of l1_regress for one design.
 * prm.s == 0 asks the library to choose the FWHT block size (see below).
 */
typedef struct {
  const void *A;       /* device, column-major n x d, leading dimension lda  */
  const void *b;       /* device, length n                                    */
  const void *A_lowp;  /* NULL, or the BF16 copy of A (then pass 2 reads it)  */
  const void *b_lowp;  /* BF16 copy of b when A_lowp != NULL                  */
  int64_t n;
  int64_t lda;
  int64_t ld_lowp;
  int32_t d;           /* 1 <= d <= 64                                        */
  int32_t pad0;
  fct_params prm;      /* as for l1_regress; s == 0: the library chooses s    */
  /* optional device outputs of the instance's intermediate results (NULL:
   * not written); they let a caller check or reuse each step */
  double *R_out;       /* (d + 1) x (d + 1) column-major, the sketch's R     */
  float *lambda_out;   /* n, the row-norm estimates of the sampling pass     */
  int64_t *idx_out;    /* idx_cap entries: the first min(S, idx_cap) are the
                        * kept rows, ascending                                */
  int64_t idx_cap;
} fct_instance;

/*
 * l1_regress_batched: the regression figure's steps 1-8 for `count`
 * independent instances of uneven n and d, all of element type dt
 * (FCT_F32 or FCT_F64).  No host synchronization happens inside the batch:
 * the whole sequence (every instance's sketch, QR, row-norm pass, selection
 * and gather, then one launch that solves all coresets, one workgroup per
 * instance) is captured into a HIP graph on the context's stream (instances
 * spread over four forked streams) and replayed on later calls with the same
 * instances, sizes and scratch; if capture is refused the sequence runs
 * eagerly.
 * Block size: for instances with prm.s == 0 the library takes the choice of
 *   the paper's experiments for FCT1 (section "Numerical experiments"),
 *   s = ceil(2 d ln d) rounded up to a power of two, at least 64 and at most
 *   1024; s_used reports it.  The rule depends on d only, so the same batch
 *   gets the same transform on every run and every device (s changes Pi1;
 *   a choice by timing would not).
 * eps: default expected coreset size s_out = ceil(20 q / eps) when prm.s_out <= 0.
 * Outputs (host): x[off_i .. off_i + d_i) with off_i = sum_{k<i} d_k;
 *   obj, S, s_used, status: count entries each, any may be NULL except status.
 *   status[i]: FCT_OK, FCT_ERR_CAPACITY (S_i > 2 s_out + 8 sqrt(s_out) + 1024;
 *   x not valid), FCT_ERR_RANK_DEFICIENT (singular coreset system) or
 *   FCT_ERR_HIP (the solver's wait timed out).
 * Returns FCT_OK if every instance succeeded, else the first failing status
 * (or a context-wide FCT_ERR_NONFINITE / FCT_ERR_RANK_DEFICIENT flagged by a
 * sketch).
 */
int l1_regress_batched(fct_ctx *ctx, const fct_instance *inst, int32_t count, fct_dtype dt,
                       double eps, double *x, double *obj, int64_t *S, int32_t *s_used,
                       int32_t *status);

/*
 * l1_select: steps 6-7 alone, from row-norm estimates already computed
 * (l1_sample_probs): p_i = min{1, s_out lambda_i / sum_lambda} in FP64 and
 * row i kept iff its stream-3 word is below floor(p_i 2^32).  Several draws
 * from one sampling pass use different seeds.
 *   lambda: device FP32 [n]; sum_lambda: device FP64 scalar.
 *   idx: device int64 [cap], ascending; w: device FP64 [cap], 1/p_i.
 *   S: host, realised count; FCT_ERR_CAPACITY when S > cap (first cap written).
 */
int l1_select(fct_ctx *ctx, const float *lambda, const double *sum_lambda, int64_t n,
              int64_t s_out, uint64_t seed, int64_t cap, int64_t *idx, double *w, int64_t *S);

/*
 * Several coresets from one sampling pass (the large-scale evaluation of
 * section "Empirical Evaluation" computes many approximate solutions in a
 * single pass over the data), drawn in one of two ways:
 *   FCT_SAMPLE_BERNOULLI: step 7 as l1_select, draw k keeping row i iff its
 *     stream-3 word of instance k is below floor(p_i 2^32);
 *   FCT_SAMPLE_REPLACE: exactly s_out rows drawn independently with
 *     replacement with probabilities lambda_i / sum lambda (the caption of
 *     the regression figure): sample j of draw k takes the row i whose
 *     interval [C_(i-1), C_i) of the running sums of lambda holds u C_n,
 *     u = (w + 1/2) / 2^32 with w its stream-4 word of instance k, and weight
 *     C_n / (s_out lambda_i).  The running sums are FP64 over 256-row blocks
 *     and their prefix; a target within rounding of a block's end takes the
 *     block's last row with lambda > 0.
 */
enum { FCT_SAMPLE_BERNOULLI = 0, FCT_SAMPLE_REPLACE = 1 };

/*
 * l1_select_draw: draw `draw` (>= 0) of either kind from row-norm estimates
 * already computed (l1_sample_probs).
 *   lambda: device FP32 [n]; sum_lambda: device FP64 scalar (Bernoulli only;
 *     the draw with replacement forms its own running sums).
 *   idx: device int64 [cap]; w: device FP64 [cap]: Bernoulli: the kept rows
 *     ascending and 1/p_i; with replacement: the s_out samples in sample
 *     order (a row drawn twice appears twice) and their weights (cap >= s_out).
 *   S: host, the count; FCT_ERR_CAPACITY when S > cap (first cap written).
 */
int l1_select_draw(fct_ctx *ctx, const float *lambda, const double *sum_lambda, int64_t n,
                   int64_t s_out, uint64_t seed, int32_t draw, int32_t mode, int64_t cap,
                   int64_t *idx, double *w, int64_t *S);

/*
 * l1_regress_multi: the regression figure's steps 1-5 once (one sketch, one
 * pass over X for lambda), then K draws (k = 0 .. K-1) of step 6-7 of the
 * given kind, each gathered into its own coreset, and the K coreset solves
 * of step 8 in one launch (one workgroup per draw).  Arguments as l1_regress
 * (FP32 or FP64 data, d <= 64, eps sets s_out when prm->s_out <= 0).
 * Outputs (host): x[k d .. k d + d), obj[k] (may be NULL), S[k] (may be
 * NULL), status[k] as l1_regress_batched's.
 * Returns FCT_OK if every draw succeeded, else the first failing status.
 */
int l1_regress_multi(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d, int64_t lda,
                     fct_dtype dt, double eps, const fct_params *prm, int32_t K, int32_t mode,
                     double *x, double *obj, int64_t *S, int32_t *status);

/*
 * l1_regress_mrhs: multiple l1 regression (section "Generalizing to Multiple
 * l1 Regression", Theorem FCRmult): min_W ||A W - B||_1 for B with k columns.
 * X = [A, -B] (q = d + k columns) is sketched and sampled once, as in the
 * regression figure with q in place of d + 1, and the k weighted regressions
 * min_w ||D (A w - B_j)||_1 are solved on the one coreset in one launch (one
 * workgroup per column).
 *   A: device, column-major n x d (lda >= n); B: device, column-major n x k
 *     (ldb >= n), same element type dt (F32 or F64); d <= 64, d + k <= 88.
 *   eps: s_out = ceil(20 q / eps) when prm->s_out <= 0.
 *   W: host FP64 d x k, column-major (column j solves right-hand side j);
 *   obj: host k or NULL, coreset objectives; S: host or NULL, coreset size;
 *   status: host k, as l1_regress_batched's.
 *   R_out, lambda_out: device or NULL: R of the sketch ((d + k) x (d + k),
 *     column-major, FP64) and the row-norm estimates (n, FP32).
 */
int l1_regress_mrhs(fct_ctx *ctx, const void *A, const void *B, int64_t n, int32_t d, int32_t k,
                    int64_t lda, int64_t ldb, fct_dtype dt, double eps, const fct_params *prm,
                    double *W, double *obj, int64_t *S, int32_t *status, double *R_out,
                    float *lambda_out);

/*
 * l1_subspace: l1-norm subspace approximation (section "Application to l1
 * norm Subspace Approximation", Theorem L1Sub): the best (d - 1)-dimensional
 * subspace for the n points (rows of A) by d constrained regressions
 * min_{w: w_j = -1} ||A w||_1, one coreset of X = A for all of them (the
 * regression figure with b empty), the d solves in one launch, then
 * err_j = ||A w_j||_1 over all rows and j* = argmin_j err_j.  The points
 * projected onto the answer are A with column j* replaced by A w (w = w_j*
 * with its -1 entry set to 0).
 *   A: device, column-major n x d, 2 <= d <= 64, F32 or F64.
 *   W: host FP64 d x d, column-major: column j is w_j (W_jj = -1).
 *   err: host d, FP64; j_star: host; S: host or NULL, coreset size;
 *   status: host d, per regression.
 *   R_out, lambda_out: device or NULL: R of the sketch of A (d x d) and the
 *     row-norm estimates (n, FP32).
 */
int l1_subspace(fct_ctx *ctx, const void *A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
                double eps, const fct_params *prm, double *W, double *err, int32_t *j_star,
                int64_t *S, int32_t *status, double *R_out, float *lambda_out);

/* ---- supporting calls (diagnostics and data preparation) ---------------- */

/*
 * fct_lowp_residual: the residual form of the design for the BF16 sampling
 * pass.  The row-norm estimates of the regression figure's steps 4-5 depend
 * on X only through X R^-1, which a change of basis T leaves alone:
 * (X T)(R T)^-1 = X R^-1.  With T = [I x0; 0 1] and x0 the least-squares
 * solution of the sketched problem (R_AA x0 = -r_Ab for R = [R_AA r_Ab;
 * 0 r_bb], the R of fct_sketch with b), X T = [A, -r0] with r0 = b - A x0:
 * the column rounded to BF16 then carries the residual, usually far smaller
 * than b, so its rounding error shrinks with it.  Pass the BF16 copy of A,
 * r_lowp as its b, and R_res as R to l1_sample_probs (l1_regress forms its
 * own R and does not take this form).
 *   A, b: device, column-major n x d and n, element type dt (F32 or F64).
 *   R: device FP64 (d+1) x (d+1), column-major, from fct_sketch with b.
 *   r_lowp: device BF16 [n]: r0 formed in FP64, rounded to FP32 and then to
 *     the nearest BF16 (ties to even).
 *   R_res: device FP64 (d+1) x (d+1), column-major: R T, its last column
 *     R_AA x0 + r_Ab formed explicitly (zero up to rounding).
 * d <= 64.  Enqueued on the context's stream; no synchronization.
 */
int fct_lowp_residual(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d,
                      int64_t lda, fct_dtype dt, const double *R, uint16_t *r_lowp,
                      double *R_res);

/* words: device uint32 [4 * count], the Philox4x32-10 words of calls
 * idx0 .. idx0 + count - 1 of `stream` (0..6) under `seed`, instance 0. */
int fct_rng_words(fct_ctx *ctx, uint32_t stream, uint64_t seed, uint64_t idx0, int64_t count,
                  uint32_t *words);

/* Per padded row j in [j0, j0 + count) of a sketch with block size s:
 * bucket and Cauchy of its H-half position 2 s floor(j/s) + (j mod s)
 * (bucket_h, cauchy_h) and of its I-half position (+ s) (bucket_i,
 * cauchy_i), and its sign (stream 1), as the sketch kernels compute them.
 * Device outputs, each of length count; sign is +1/-1 as int8. */
int fct_pi1_streams(fct_ctx *ctx, uint64_t seed, int32_t r1, int32_t s, uint64_t j0, int64_t count,
                    int32_t *bucket_h, float *cauchy_h, int32_t *bucket_i, float *cauchy_i,
                    int8_t *sign);

/* In-place normalized Walsh-Hadamard transform (Sylvester order) of every
 * consecutive block of s values of x (device FP32 [nblocks * s]), with the
 * kernel the sketch uses.  s power of two in [2, 4096]. */
int fct_fwht(fct_ctx *ctx, float *x, int64_t nblocks, int32_t s);

/* Kernel timing: enable != 0 starts recording HIP events around every
 * pass-1 kernel (kind 0), pass-2 kernel (kind 1), step-8 solve sequence
 * (kind 2), FCT2 FJLT kernel (kind 3) and FCT2 Cauchy contraction (kind 4)
 * launched on the context's stream (up to 512 of each; counts are
 * reset); 0 stops.  fct_profile_read waits for the stream and returns the
 * summed device milliseconds and the number of launches of `kind`. */
int fct_profile(fct_ctx *ctx, int enable);
int fct_profile_read(fct_ctx *ctx, int kind, double *total_ms, int64_t *count);

/* Plan options of a context, for benchmarks and tests (the defaults need no
 * call).  FCT_OPT_PASS1_KERNEL: FCT_P1_AUTO (default), FCT_P1_WAVE (the
 * wave-level kernel with a random table), FCT_P1_OWNER (the bucket-owner
 * kernel, FP32 with s <= 1024), FCT_P1_TILE (the workgroup-tile kernel); a
 * choice that does not fit a shape falls back to the automatic one.
 * FCT_OPT_PASS1_WGS_PER_CU: workgroups per CU the pass-1 grids aim for (>= 1).
 * FCT_OPT_PASS1_TILE_THREADS: 256, 512 or 1024.  FCT_OPT_PASS2_WGS: cap of the
 * FP32/BF16 pass-2 grid (0 = default).  FCT_OPT_SOLVE_WGS, FCT_OPT_SOLVE_ROWS:
 * workgroups of the coreset solve, or coreset rows per workgroup (0 =
 * default).  FCT_OPT_FCT2_OVERLAP: 1 runs FCT2's Cauchy contraction of each
 * eighth of the rows on a second stream while a capped FJLT grid works on
 * the next eighth (measured slower than the default on MI355X: the two
 * kernels contend for the same CUs); 0 (default) runs the two kernels one
 * after the other, each over all rows.  Returns
 * FCT_ERR_BAD_ARG for an unknown option or value.
 */
enum {
  FCT_OPT_PASS1_KERNEL = 1,
  FCT_OPT_PASS1_WGS_PER_CU = 2,
  FCT_OPT_PASS1_TILE_THREADS = 3,
  FCT_OPT_PASS2_WGS = 4,
  FCT_OPT_SOLVE_WGS = 5,
  FCT_OPT_SOLVE_ROWS = 6,
  FCT_OPT_FCT2_OVERLAP = 7
};
enum { FCT_P1_AUTO = 0, FCT_P1_WAVE = 1, FCT_P1_OWNER = 2, FCT_P1_TILE = 3 };
int fct_set_option(fct_ctx *ctx, int option, int64_t value);

/* BF16 copy (round to nearest even) of a device FP32 array. */
int fct_to_bf16(fct_ctx *ctx, const float *x, int64_t count, uint16_t *y);

/* out[j] = sum_i |(A W)_ij - B_ij| in FP64 for the k columns of W (host FP64
 * d x k, column-major; d, k <= 64); B: device n x k (ldb >= n) or NULL. */
int fct_l1_objectives(fct_ctx *ctx, const void *A, const void *B, int64_t n, int32_t d, int32_t k,
                      int64_t lda, int64_t ldb, fct_dtype dt, const double *W, double *out);

/* sum_i |A_i x - b_i| over all n rows (device reduction, FP64 result).
 * x: host double[d]; out: host double. */
int fct_l1_objective(fct_ctx *ctx, const void *A, const void *b, int64_t n, int32_t d, int64_t lda,
                     fct_dtype dt, const double *x, double *out);

/* Weighted l1 solve of step 8 alone: x = argmin sum_k w_k |At_k x - bt_k|
 * on a device coreset (At: S x d column-major, ld = ldat; bt, w device).
 * x: host double[d]; obj: host double or NULL. */
int l1_solve(fct_ctx *ctx, const void *At, const void *bt, const double *w, int64_t S, int32_t d,
             int64_t ldat, fct_dtype dt, int32_t iters, double *x, double *obj);

#ifdef __cplusplus
}
#endif
#endif /* FCTL1_H */
