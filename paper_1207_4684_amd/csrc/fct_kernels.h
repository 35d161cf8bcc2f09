// Internal interface between the C ABI (fctl1_api.hip) and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fctl1 {

struct Pass1Args {
  const void* A;
  const void* b;       // NULL when X = A; else the k = q - d columns of B, X = [A, -B]
  int64_t lda;
  int64_t ldb;         // leading dimension of B
  int64_t n;           // rows
  int64_t n_pad;       // s * ceil(n / s)
  int64_t rows_per_range;
  int32_t d;           // columns of A
  int32_t q;           // columns of X
  int32_t s;
  int32_t log2s;
  int32_t r1;
  int32_t c;           // columns per slice (last slice may be narrower)
  uint64_t seed;
  uint32_t instance;
  int32_t sign_flip;
  int64_t row0g;       // global index of local row 0 (random streams are indexed globally)
  void* partials;      // [nranges][q][r1] of the input type
  const uint4* tab_keys;  // wave kernel: per row, H bucket | sign of D(j) << 15 | I bucket << 16
  const float4* tab_c;    // wave kernel: per row, (4 C_H / sqrt(s), 4 C_I), two rows per float4
  float scale_h;          // owner kernel: 4 / sqrt(s), the H-half factor
  int32_t bucket_span;    // owner kernel: buckets per workgroup (<= 1024; grid z covers r1)
};

struct Pass1Plan {
  int kind;            // 0: workgroup-tile kernel, 1: wave-level kernel (FP32, s <= 2048),
                       // 2: bucket-owner kernel (FP32, s <= 1024; deterministic)
  bool vec_ok;         // 16-byte aligned columns (wave kernel float4 loads)
  int threads;
  int rpt;             // rows per thread per chunk
  int c;
  int nslices;
  int nranges;
  int nbranges;        // owner kernel: bucket ranges (grid z)
  int bucket_span;     // owner kernel: buckets per range
  int64_t rows_per_range;
  size_t lds;
};

hipError_t launch_pass1(const Pass1Args& a, const Pass1Plan& p, bool f64, hipStream_t st);
// Row stride (doubles) of the wave kernels' LDS accumulator for a slice of c
// columns.  A lane group adds 4 adjacent columns of 16 random buckets; with a
// stride that is a multiple of 4 the buckets' first columns fall on a few
// banks (an FP64 LDS atomic measured 79 clocks at stride 8 against 27 at
// stride 7), so even widths above 2 are padded by one column.
__host__ __device__ inline int pass1_acc_stride(int c) { return (c > 2 && !(c & 1)) ? c + 1 : c; }
// LDS bytes of the wave kernels: accumulator of r1 rows x `stride` doubles,
// per-wave tables, and the exchange buffer for s > 256.
size_t pass1_wave_lds(int r1, int stride, int s);
int pass1_wave_rows_quantum();
// whether the wave form for block size s reads the signs of D from the table
// (s > 256) or draws them itself
bool pass1_wave_signs_in_table(int s);
// rows of the wave kernel's random table for n_pad padded rows (whole tiles)
int64_t pi1_table_rows(int64_t n_pad);
// the table: keys[rows / 4] (uint4), cc[rows / 2] (float4); rows a multiple of 4
hipError_t launch_pi1_table(uint64_t seed, uint32_t instance, int64_t row0g, int64_t rows, int s,
                            int r1, int sign_flip, uint4* keys, float4* cc, hipStream_t st);
hipError_t launch_pass1_wave(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st);
// Bucket-owner form (pass1_owner.hip): columns per slice for a bucket span,
// its LDS bytes, the tile height (rows per workgroup step) and the launch.
int pass1_owner_max_cols(int span);
size_t pass1_owner_lds(int span, int c);
int pass1_owner_tile_rows();
hipError_t launch_pass1_owner(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st);
// FCT2: the FJLT blocks (fct2_fjlt_kernel) and the Cauchy contraction.
constexpr int kFct2MaxS = 256;
struct Fct2Args {
  const void* A;
  const void* b;     // NULL when X = A; else X = [A, -b]
  int64_t lda;
  int64_t n;
  int32_t d;
  int32_t q;
  int32_t s;         // rows G keeps per block, 1 <= s <= min(t, kFct2MaxS)
  int32_t log2t;     // block size t = 2^log2t, 6 <= log2t <= 12
  int64_t nb;        // blocks, ceil(n / t)
  int64_t beta0;     // first block of this launch, which covers nbl blocks
  int64_t nbl;
  int64_t fjlt_grid; // workgroups of the FJLT launch (0: one per block)
  int64_t row0g;     // global row of local row 0 (a multiple of t)
  uint64_t seed;
  uint32_t instance;
  double* Z;         // (nb s) x zq row-major, G z per block
  int32_t zq;        // row stride of Z: q rounded up to whole slices
  int32_t r1;
  int64_t K;         // nb s, columns of C
  int64_t kc;        // columns of C per chunk (a multiple of 4)
  int64_t mbase;     // this launch's columns of C: [mbase, mend), mbase a multiple of 4,
  int64_t mend;      //   in chunks chunk0 .. chunk0 + nchunks - 1 of the partials
  int32_t chunk0;
  int32_t nchunks;
  double scale;      // 8 / r1 sqrt(pi t / (2 s))
  double* partials;  // [nchunks][q][r1]
};
// columns per slice of the contraction for q columns (8, 17 or 33)
int fct2_slice_width(int q);
hipError_t launch_fct2_fjlt(const Fct2Args& a, bool f64, hipStream_t st);
hipError_t launch_fct2_cauchy(const Fct2Args& a, bool f64, hipStream_t st);
// y_f64 < 0: Y has the partials' type; else FP64 (1) or FP32 (0)
hipError_t launch_reduce_partials(const void* part, int nranges, int r1, int q, void* Y,
                                  double* Yd, int* flag, bool f64, hipStream_t st,
                                  int y_f64 = -1);
hipError_t launch_rng_words(uint32_t stream, uint64_t seed, uint64_t idx0, int64_t count,
                            uint32_t* out, hipStream_t st);
hipError_t launch_pi1_streams(uint64_t seed, uint32_t r1, int log2s, uint64_t j0, int64_t count,
                              int32_t* bh, float* ch, int32_t* bi, float* ci, int8_t* sg,
                              hipStream_t st);
hipError_t launch_fwht(float* x, int64_t nblocks, int s, int log2s, hipStream_t st);

// QR of the FP64 sketch (tall r1 x q, column-major, ld = r1) by a tree of
// Householder panel factorizations.  work must hold qr_work_doubles(r1, q).
size_t qr_work_doubles(int r1, int q);
// rank_tol: R is rank deficient when some |R_jj| <= rank_tol * ||R[:, j]||_2
// (the component of column j orthogonal to the earlier columns, relative to
// the column's own norm).
hipError_t launch_qr(const double* Y, int r1, int q, double* work, double* R, double rank_tol,
                     int* status, hipStream_t st);
// M = R^-1 Pi2 (q x r2), written row-major with row stride ldm >= r2 (zero
// padding) as FP64, and when non-NULL as FP32 (Mf), as FP32 values of its
// BF16 rounding (Mfb) and as BF16 bit patterns (Mb).
// gaussian: Pi2 of standard Gaussians (optimized regression) instead of Cauchys.
hipError_t launch_form_m(const double* R, int q, int r2, int ldm, uint64_t seed,
                         uint32_t instance, double* Md, float* Mf, float* Mfb, uint16_t* Mb,
                         int* status, hipStream_t st, bool gaussian = false);
__host__ __device__ int r2_padded(int r2);

// Pass 2: lambda and per-workgroup FP64 partial sums of lambda.
struct Pass2Args {
  const void* A;
  const void* b;       // NULL, or the q - d columns of B (X = [A, -B])
  int64_t lda;
  int64_t ldb;
  int64_t n;
  int32_t d;
  int32_t q;
  int32_t r2;
  const void* M;       // q x r2_padded row-major: FP64 for FP64 data, else FP32
                       // (the BF16-rounded values for the BF16 path)
  const uint16_t* Mb;  // same layout, BF16 bits (BF16 path)
  float* lambda;
  double* wg_sums;     // [grid]
};
enum Pass2Kind { kPass2F32 = 0, kPass2F64 = 1, kPass2BF16 = 2 };
// grid of the pass-2 kernel of `kind` for n rows (cap_override > 0 caps the
// MFMA forms' grid instead of the default); the caller sizes the per-workgroup
// sums with the same value and passes it to launch_pass2.
int pass2_grid(int64_t n, int kind, int cap_override = 0);
hipError_t launch_pass2(const Pass2Args& a, int kind, int grid, hipStream_t st);
hipError_t launch_sum_fixed(const double* parts, int count, double* out, hipStream_t st);

// Selection: p_i = min(1, s_out lambda_i / sum), keep iff word_i < floor(p_i 2^32).
struct SelectArgs {
  const float* lambda;
  const double* sum_lambda;
  int64_t n;
  double s_out;
  uint64_t seed;
  uint32_t instance;
  float* p_out;        // optional
  uint64_t* lookback;  // [grid + 1]: look-back status of each tile, then the ticket counter
  int32_t* fail;       // device flag: FCT_ERR_HIP if the look-back wait timed out
  int64_t* idx;        // [cap]
  double* w;           // [cap]
  int64_t cap;
  int64_t* S;          // device scalar
};
int select_grid(int64_t n);
hipError_t launch_select(const SelectArgs& a, hipStream_t st);
// Sampling with replacement: block sums bs [rep_blocks(n)], their prefix pre
// [rep_blocks(n)], chunk sums cs and offsets co [rep_chunks(n)] and the total
// tot [1] (built when build_cdf), then s samples of draw `instance`.
int64_t rep_blocks(int64_t n);
int64_t rep_chunks(int64_t n);
hipError_t launch_select_replace(const float* lambda, int64_t n, int64_t s, uint64_t seed,
                                 uint32_t instance, double* bs, double* pre, double* cs,
                                 double* co, double* tot, bool build_cdf, int64_t* idx, double* w,
                                 int64_t* S, hipStream_t st);
hipError_t launch_probs_only(const SelectArgs& a, hipStream_t st);

// Gather the kept rows of A and b (unscaled) into column-major outputs.
hipError_t launch_gather(const void* A, const void* b, int64_t lda, int32_t d, int32_t kb,
                         int64_t ldb, const int64_t* idx,
                         const int64_t* S, int64_t cap, void* At, void* bt, int64_t ldat, bool f64,
                         hipStream_t st);

// Step 8: weighted l1 solve by FP64 IRLS.
size_t irls_work_doubles(int64_t S, int d);
// Arguments of one IRLS solve (step 8).
struct IrlsArgs {
  const void* At;
  const void* bt;
  const double* w;
  const int64_t* S_dev;
  int64_t cap;
  int64_t ldat;
  int d;
  int iters;
  int row_target;  // coreset rows per active workgroup
  double* part;    // 2 x workgroups x pstride
  unsigned* bar;   // [0] arrival counter (zero at launch), [1] abort flag
  double* x_out;
  double* obj_out;
  int* status;
  int wg0;         // batched form with a block map: first block of the instance in its launch
  int nwg;         //   and its workgroups
};
// Batched form (all of one element type): arr is a device array of count
// instances; each has work of irls_batched_work_doubles(d, nwg) doubles and
// its barrier words at irls_batched_bar(work, d, nwg).  Without binst, block
// b solves instance b alone (nwg = 1); with it, block b works on instance
// binst[b] (workgroup b - wg0 of its nwg), and nblocks must not exceed what
// the device holds at once (irls_max_resident_wgs).  reset clears every
// instance's barrier and status first.
size_t irls_batched_work_doubles(int d, int nwg = 1);
unsigned* irls_batched_bar(double* work, int d, int nwg = 1);
int irls_max_resident_wgs(int cus);
hipError_t launch_irls_batched(const IrlsArgs* arr, int count, bool f64, hipStream_t st,
                               const int* binst = nullptr, int nblocks = 0, bool reset = true);
// Persistent cooperative IRLS: S_hint (host) sizes the grid, the device count
// S_dev (clamped to cap) is the number of rows; x_out[d], obj_out[1].
hipError_t launch_irls(const void* At, const void* bt, const double* w, const int64_t* S_dev,
                       int64_t cap, int64_t S_hint, int d, int64_t ldat, bool f64, int iters,
                       double* work, double* x_out, double* obj_out, int* status,
                       hipStream_t st, int rows_override = 0, int wgs_override = 0);

hipError_t launch_to_bf16(const float* x, int64_t count, uint16_t* y, hipStream_t st);
// x0 = -R_AA^-1 r_Ab, R_res = R T and the BF16 residual r0 = b - A x0.
hipError_t launch_lowp_residual(const void* A, const void* b, int64_t lda, int64_t n, int d,
                                bool f64, const double* R, double* x0, double* R_res, uint16_t* r,
                                hipStream_t st);
// sum_i |(A W)_ij - B_ij| for the k columns of W (B may be NULL), FP64.
hipError_t launch_l1_objectives(const void* A, const void* B, int64_t lda, int64_t ldb, int64_t n,
                                int d, int k, const double* W, bool f64, double* parts, int nparts,
                                double* out, hipStream_t st);
// Subspace approximation: per column j, the coreset without column j and column j.
hipError_t launch_drop_column(const void* At, int64_t cap, int d, const int64_t* S, void* Aj,
                              void* bj, bool f64, hipStream_t st);
hipError_t launch_l1_objective(const void* A, const void* b, int64_t lda, int64_t n, int d,
                               const double* x, bool f64, double* parts, int nparts, double* out,
                               hipStream_t st);

}  // namespace fctl1
