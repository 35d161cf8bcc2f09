// C ABI of fctl1 (declared in include/fctl1.h): argument checks, work plans,
// scratch management and the launch sequences of the FastCauchyRegression
// path (regression figure steps 1-8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fctl1.h"
#include "fct_kernels.h"

using namespace fctl1;

// Scratch of l1_sample_probs_noalloc: M = R^-1 Pi2 in its four forms and the
// per-workgroup partial sums of lambda, in a static device array (one copy
// per GPU, alive until the process ends).  Host code never uses the symbol's
// name as an address: fct_create looks up each device's copy once with
// hipGetSymbolAddress and the entry point passes that pointer.
static constexpr size_t kNoAllocBytes = 80 * 1024;
static __device__ __align__(256) unsigned char g_noalloc_scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};
}  // namespace

struct fct_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  int* flags = nullptr;         // device: [0] non-finite, [1] rank / solve status
  void* pinned = nullptr;       // host pinned staging for small readbacks
  int cus = 256;
  size_t lds_optin = 65536;
  // optional per-kernel timing with HIP events on the context stream
  static constexpr int kProfSlots = 512;
  static constexpr int kProfKinds = 5;
  bool prof_on = false;
  int prof_n[kProfKinds] = {};
  hipEvent_t* prof_ev[kProfKinds] = {};  // pairs (start, stop)
  // plan knobs (fct_set_option)
  int p1_kernel = FCT_P1_AUTO;  // pass-1 kernel choice
  int p1_threads = 256;         // workgroup-tile kernel threads
  size_t p1_lds_budget = 0;     // 0: the device's opt-in maximum
  int p1_waves_of_wgs = 1;      // workgroups per CU the pass-1 grids aim for
  int p2_wgs = 0;               // 0: default pass-2 grid cap
  int irls_wgs = 0;             // 0: solver workgroups from the coreset size
  int irls_rows = 0;            // 0: default coreset rows per solver workgroup
  int fct2_overlap = 0;         // FCT2: contraction of segment k beside the FJLT of k + 1
  static constexpr int kFct2Segs = 8;
  hipEvent_t ev_seg[kFct2Segs] = {};
  // batched form: forked streams, events, staging and the cached graph
  static constexpr int kBranches = 4;
  hipStream_t branch[kBranches] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kBranches] = {};
  void* bpinned = nullptr;
  size_t bpinned_bytes = 0;
  hipGraphExec_t bgraph = nullptr;
  std::vector<char> bsig;       // signature of the captured batch
  void* noalloc = nullptr;      // this device's copy of g_noalloc_scratch (nullptr: lookup failed)
};

namespace {

// timing brackets around one launch sequence of kind k (0 pass 1, 1 pass 2, 2 solve,
// 3 FCT2 FJLT blocks, 4 FCT2 Cauchy contraction), on the context's stream or `st`
void prof_begin(fct_ctx* c, int k, hipStream_t st = nullptr) {
  if (!c->prof_on || !c->prof_ev[k] || c->prof_n[k] >= fct_ctx::kProfSlots) return;
  (void)hipEventRecord(c->prof_ev[k][2 * c->prof_n[k]], st ? st : c->stream);
}
void prof_end(fct_ctx* c, int k, hipStream_t st = nullptr) {
  if (!c->prof_on || !c->prof_ev[k] || c->prof_n[k] >= fct_ctx::kProfSlots) return;
  (void)hipEventRecord(c->prof_ev[k][2 * c->prof_n[k] + 1], st ? st : c->stream);
  ++c->prof_n[k];
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return FCT_ERR_HIP; \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
size_t esize(fct_dtype dt) { return dt == FCT_F64 ? 8 : (dt == FCT_BF16 ? 2 : 4); }

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(char* b) : base(b) {}
  template <typename T> T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Size-only pass of a Carve sequence.
struct Measure {
  size_t off = 0;
  template <typename T> void take(size_t count) {
    off = (off + 255) & ~size_t(255);
    off += count * sizeof(T);
  }
};

int ensure_scratch(fct_ctx* c, size_t bytes) {
  if (bytes <= c->scratch_bytes) return FCT_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->bgraph) {  // a captured batch points into the old arena
    (void)hipGraphExecDestroy(c->bgraph);
    c->bgraph = nullptr;
    c->bsig.clear();
  }
  if (c->scratch) HIP_TRY(hipFree(c->scratch));
  c->scratch = nullptr;
  c->scratch_bytes = 0;
  size_t want = bytes + bytes / 4 + (1 << 20);
  if (hipMalloc(&c->scratch, want) != hipSuccess) {
    c->scratch = nullptr;
    return FCT_ERR_OOM;
  }
  c->scratch_bytes = want;
  return FCT_OK;
}

Pass1Plan make_wave_plan(const fct_ctx* c, int64_t n_pad, int q, int s, int r1, int* err) {
  Pass1Plan p{};
  p.kind = 1;
  p.threads = 512;
  p.rpt = 1;
  *err = 0;
  const size_t budget = c->p1_lds_budget ? c->p1_lds_budget : c->lds_optin;
  const size_t fixed = pass1_wave_lds(r1, 0, s) + 16;
  const size_t per_col = (size_t)r1 * sizeof(double);
  if (budget <= fixed + per_col) {
    *err = 1;
    return p;
  }
  int cmax = (int)((budget - fixed) / per_col);
  // the padded accumulator row (pass1_acc_stride) must fit too
  while (cmax > 1 && (size_t)pass1_acc_stride(cmax) * per_col > budget - fixed) --cmax;
  if (cmax > q) cmax = q;
  // widest slices: every slice re-reads the random table and re-runs the
  // per-tile set-up, which costs more than the lanes a width that is not a
  // multiple of 4 leaves idle (their adds are masked off)
  p.nslices = (q + cmax - 1) / cmax;
  p.c = (q + p.nslices - 1) / p.nslices;
  p.nslices = (q + p.c - 1) / p.c;
  p.lds = pass1_wave_lds(r1, pass1_acc_stride(p.c), s);
  int per_cu = (int)((size_t)(160 * 1024) / p.lds);
  if (per_cu < 1) per_cu = 1;
  const int64_t target = (int64_t)c->cus * per_cu * c->p1_waves_of_wgs;
  int64_t nranges = target / p.nslices;
  if (nranges < 1) nranges = 1;
  const int64_t min_ranges = (n_pad + 262143) / 262144;
  if (nranges < min_ranges) nranges = min_ranges;
  const int64_t quantum = pass1_wave_rows_quantum();
  int64_t rpr = (n_pad + nranges - 1) / nranges;
  rpr = (rpr + quantum - 1) / quantum * quantum;
  p.rows_per_range = rpr;
  p.nranges = (int)((n_pad + rpr - 1) / rpr);
  return p;
}

// Bucket-owner plan: grid (row ranges, column slices, bucket ranges).
Pass1Plan make_owner_plan(const fct_ctx* c, int64_t n_pad, int q, int r1) {
  Pass1Plan p{};
  p.kind = 2;
  p.threads = 512;
  p.rpt = 1;
  p.nbranges = (r1 + 1023) / 1024;
  p.bucket_span = (r1 + p.nbranges - 1) / p.nbranges;
  const int cmax = pass1_owner_max_cols(p.bucket_span);
  p.nslices = (q + cmax - 1) / cmax;
  p.c = (q + p.nslices - 1) / p.nslices;
  p.nslices = (q + p.c - 1) / p.c;
  p.lds = pass1_owner_lds(p.bucket_span, p.c);
  const int64_t tile = pass1_owner_tile_rows();
  const int64_t ntiles = (n_pad + tile - 1) / tile;
  int64_t nranges = (int64_t)c->cus * c->p1_waves_of_wgs / ((int64_t)p.nslices * p.nbranges);
  if (nranges < 1) nranges = 1;
  if (nranges > ntiles) nranges = ntiles;
  int64_t tpr = (ntiles + nranges - 1) / nranges;
  // the kernel's per-bucket accumulators are FP32: at most 16 tiles per
  // range, unless that takes more than 4096 ranges (64 tiles at n = 2^31)
  const int64_t tpr_cap = std::max<int64_t>(16, (ntiles + 4095) / 4096);
  if (tpr > tpr_cap) tpr = tpr_cap;
  p.rows_per_range = tpr * tile;
  p.nranges = (int)((ntiles + tpr - 1) / tpr);
  return p;
}

// Pass-1 kernel for a sketch.  FP32 data with s <= 1024 takes the
// bucket-owner kernel when r1 <= 1024 (one workgroup holds every bucket) or
// when the caller asks for a deterministic sketch; other shapes take the
// wave-level kernel (FP32, s <= 2048) or the workgroup-tile kernel, whose LDS
// atomic adds make the sums reproducible to rounding only.  *err = 1: no
// kernel fits; *err = 2: a deterministic sketch of this shape is not offered.
Pass1Plan make_pass1_plan(const fct_ctx* c, int64_t n_pad, int q, int s, int r1, size_t es,
                          uint32_t flags, int* err) {
  *err = 0;
  const bool owner_ok = es == sizeof(float) && s <= 1024;
  const bool det = (flags & FCT_FLAG_DETERMINISTIC) != 0;
  if (det && !owner_ok) {
    *err = 2;
    return Pass1Plan{};
  }
  if (owner_ok && (det || c->p1_kernel == FCT_P1_OWNER ||
                   (c->p1_kernel == FCT_P1_AUTO && r1 <= 1024)))
    return make_owner_plan(c, n_pad, q, r1);
  if (es == sizeof(float) && s <= 2048 && r1 <= 32768 && c->p1_kernel != FCT_P1_TILE) {
    Pass1Plan w = make_wave_plan(c, n_pad, q, s, r1, err);
    if (!*err) return w;
  }
  Pass1Plan p{};
  p.kind = 0;
  p.threads = c->p1_threads;
  const int chunk = s > p.threads ? s : p.threads;
  p.rpt = chunk / p.threads;
  const size_t tp = (size_t)chunk + chunk / 16;
  const size_t budget = c->p1_lds_budget ? c->p1_lds_budget : c->lds_optin;
  const size_t fixed = (size_t)(chunk / 32) * 4 + 256;
  const size_t per_col = (size_t)r1 * es + tp * es;
  *err = 0;
  if (budget <= fixed + per_col) {
    *err = 1;
    return p;
  }
  int cmax = (int)((budget - fixed) / per_col);
  if (cmax > q) cmax = q;
  p.nslices = (q + cmax - 1) / cmax;
  p.c = (q + p.nslices - 1) / p.nslices;
  p.nslices = (q + p.c - 1) / p.c;  // every slice non-empty
  p.lds = (size_t)r1 * p.c * es + (size_t)p.c * tp * es + fixed;
  int per_cu = (int)((size_t)(160 * 1024) / p.lds);
  if (per_cu < 1) per_cu = 1;
  const int64_t target = (int64_t)c->cus * per_cu * c->p1_waves_of_wgs;
  int64_t nranges = target / p.nslices;
  if (nranges < 1) nranges = 1;
  const int64_t min_ranges = (n_pad + 262143) / 262144;  // bound rows summed per partial
  if (nranges < min_ranges) nranges = min_ranges;
  const int64_t max_ranges = (n_pad + chunk - 1) / chunk;
  if (nranges > max_ranges) nranges = max_ranges;
  int64_t rpr = (n_pad + nranges - 1) / nranges;
  rpr = (rpr + chunk - 1) / chunk * chunk;
  p.rows_per_range = rpr;
  p.nranges = (int)((n_pad + rpr - 1) / rpr);
  return p;
}

int check_common(const fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda) {
  if (!c || !A || n < 1 || d < 1 || lda < n) return FCT_ERR_BAD_ARG;
  return FCT_OK;
}

// pinned staging layout: [0, 1024) results, [1024, 2048) counts, [2048, 3072)
// host-to-device arguments, [3072, 3080) status flags
constexpr size_t kPinFlags = 3072;

int read_flags(fct_ctx* c) {
  int h[2] = {0, 0};
  char* stage = (char*)c->pinned + kPinFlags;
  HIP_TRY(hipMemcpyAsync(stage, c->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(h, stage, sizeof(h));
  HIP_TRY(hipMemsetAsync(c->flags, 0, 2 * sizeof(int), c->stream));
  if (h[0]) return FCT_ERR_NONFINITE;
  if (h[1]) return h[1];
  return FCT_OK;
}

// ---- internal steps -------------------------------------------------------

struct SketchBufs {
  void* partials;
  double* Yd;
  double* qrwork;
};

template <typename C>
void carve_sketch(C& cv, const Pass1Plan& p, int64_t n_pad, int q, int r1, size_t es, bool want_r) {
  cv.template take<char>((size_t)p.nranges * q * r1 * (p.kind == 2 ? sizeof(float) : es));
  cv.template take<double>((size_t)r1 * q);
  if (p.kind == 1) {
    const int64_t rows = pi1_table_rows(n_pad);
    cv.template take<uint4>((size_t)rows / 4);
    cv.template take<float4>((size_t)rows / 2);
  }
  if (want_r) cv.template take<double>(qr_work_doubles(r1, q));
}

int run_sketch(fct_ctx* c, Carve& cv, const void* A, int64_t n, int32_t d, int64_t lda,
               fct_dtype dt, const void* b, int32_t s, int32_t r1, uint64_t seed, uint32_t flags,
               void* Y, double* R, double** Yd_out, const Pass1Plan& p, int64_t row0g = 0,
               int32_t kb = 1, int64_t ldb = 0) {
  const int q = d + (b ? kb : 0);
  const int64_t n_pad = (n + s - 1) / s * s;
  const size_t es = esize(dt);
  void* partials = cv.take<char>((size_t)p.nranges * q * r1 * (p.kind == 2 ? sizeof(float) : es));
  double* Yd = cv.take<double>((size_t)r1 * q);
  uint4* tab_keys = nullptr;
  float4* tab_c = nullptr;
  if (p.kind == 1) {
    const int64_t rows = pi1_table_rows(n_pad);
    tab_keys = cv.take<uint4>((size_t)rows / 4);
    tab_c = cv.take<float4>((size_t)rows / 2);
  }
  Pass1Args a{};
  a.A = A;
  a.b = b;
  a.lda = lda;
  a.ldb = ldb > 0 ? ldb : n;
  a.n = n;
  a.n_pad = n_pad;
  a.rows_per_range = p.rows_per_range;
  a.d = d;
  a.q = q;
  a.s = s;
  a.log2s = ilog2(s);
  a.r1 = r1;
  a.c = p.c;
  a.seed = seed;
  a.instance = 0;
  a.sign_flip = (flags & FCT_FLAG_NO_SIGN_FLIP) ? 0 : 1;
  a.row0g = row0g;
  a.partials = partials;
  a.tab_keys = tab_keys;
  a.tab_c = tab_c;
  a.scale_h = 4.0f / sqrtf((float)s);
  a.bucket_span = p.bucket_span;
  const bool vec_ok = (lda % 4 == 0) && (((uintptr_t)A & 15) == 0) &&
                      (!b || (((uintptr_t)b & 15) == 0)) && (kb <= 1 || a.ldb % 4 == 0);
  prof_begin(c, 0);
  if (p.kind == 2) {
    HIP_TRY(launch_pass1_owner(a, p, vec_ok, c->stream));
  } else if (p.kind == 1) {
    HIP_TRY(launch_pi1_table(seed, 0, row0g, pi1_table_rows(n_pad), s, r1,
                             pass1_wave_signs_in_table(s) ? a.sign_flip : 0, tab_keys, tab_c,
                             c->stream));
    HIP_TRY(launch_pass1_wave(a, p, vec_ok, c->stream));
  } else {
    HIP_TRY(launch_pass1(a, p, dt == FCT_F64, c->stream));
  }
  prof_end(c, 0);
  HIP_TRY(launch_reduce_partials(partials, p.nranges, r1, q, Y, Yd, c->flags + 0,
                                 dt == FCT_F64 && p.kind != 2, c->stream));
  if (R) {
    double* work = cv.take<double>(qr_work_doubles(r1, q));
    const double rank_tol = dt == FCT_F64 ? 1e-13 : 1e-5;
    HIP_TRY(launch_qr(Yd, r1, q, work, R, rank_tol, c->flags + 1, c->stream));
  }
  if (Yd_out) *Yd_out = Yd;
  return FCT_OK;
}

// ---- FCT2 -------------------------------------------------------------------

struct Fct2Plan {
  int log2t;
  int64_t nb, K, kc;
  int nchunks, zq;
  int nseg;       // segments of blocks (the FJLT of one overlaps the contraction of another)
  int64_t bseg;   // blocks per segment; bseg * s is a multiple of 4 when nseg > 1
};

// segmented: the rows are split into eight segments so that the contraction of
// one can run beside the FJLT of the next (FCT_OPT_FCT2_OVERLAP)
Fct2Plan make_fct2_plan(int64_t n, int q, int t, int s, int r1, bool segmented) {
  Fct2Plan p{};
  p.log2t = ilog2(t);
  p.nb = (n + t - 1) / t;
  p.K = p.nb * s;
  const int qc = fct2_slice_width(q);
  p.zq = (q + qc - 1) / qc * qc;
  // about 4096 workgroups of 256 rows of C in all, chunks of at least 64 columns
  const int64_t per = (int64_t)((r1 + 255) / 256) * (p.zq / qc);
  int64_t nch = (4096 + per - 1) / per;
  const int64_t most = (p.K + 63) / 64;
  if (nch > most) nch = most;
  if (nch < 1) nch = 1;
  p.kc = ((p.K + nch - 1) / nch + 3) / 4 * 4;
  p.nseg = 1;
  p.bseg = p.nb;
  if (segmented && p.nb >= 8 * 64) {
    p.bseg = ((p.nb + fct_ctx::kFct2Segs - 1) / fct_ctx::kFct2Segs + 3) / 4 * 4;
    p.nseg = (int)((p.nb + p.bseg - 1) / p.bseg);
  }
  p.nchunks = 0;
  for (int k = 0; k < p.nseg; ++k) {
    const int64_t m0 = k * p.bseg * s;
    const int64_t m1 = std::min(p.K, (k + 1) * p.bseg * s);
    p.nchunks += (int)((m1 - m0 + p.kc - 1) / p.kc);
  }
  return p;
}

template <typename C>
void carve_fct2(C& cv, const Fct2Plan& p, int q, int r1, bool want_r) {
  cv.template take<double>((size_t)p.K * p.zq);
  cv.template take<double>((size_t)p.nchunks * r1 * q);
  cv.template take<double>((size_t)r1 * q);
  if (want_r) cv.template take<double>(qr_work_doubles(r1, q));
}

int batch_ensure_aux(fct_ctx* c, size_t pinned_bytes);

int check_fct2_args(const fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda,
                    fct_dtype dt, const void* b, int32_t t, int32_t s, int32_t r1, bool want_r) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  const int q = d + (b ? 1 : 0);
  if (dt != FCT_F32 && dt != FCT_F64) return FCT_ERR_BAD_ARG;
  if (!is_pow2(t) || t < 64 || t > 4096) return FCT_ERR_BAD_ARG;
  if (s < 1 || s > t || s > kFct2MaxS) return FCT_ERR_BAD_ARG;
  if (r1 < q || r1 > 65536) return FCT_ERR_BAD_ARG;
  if (want_r && q > 88) return FCT_ERR_BAD_ARG;
  if ((n + t - 1) / t > 0x7FFFFFFF) return FCT_ERR_BAD_ARG;
  return FCT_OK;
}

// Y = Pi1 X with FCT2 (X = [A, -b] when b is given); R of its QR when R != NULL.
int run_fct2(fct_ctx* c, Carve& cv, const void* A, int64_t n, int32_t d, int64_t lda,
             fct_dtype dt, const void* b, int32_t t, int32_t s, int32_t r1, uint64_t seed,
             void* Y, double* R, const Fct2Plan& p) {
  const int q = d + (b ? 1 : 0);
  Fct2Args a{};
  a.A = A;
  a.b = b;
  a.lda = lda;
  a.n = n;
  a.d = d;
  a.q = q;
  a.s = s;
  a.log2t = p.log2t;
  a.nb = p.nb;
  a.row0g = 0;
  a.seed = seed;
  a.instance = 0;
  a.Z = cv.take<double>((size_t)p.K * p.zq);
  a.zq = p.zq;
  a.r1 = r1;
  a.K = p.K;
  a.kc = p.kc;
  a.nchunks = p.nchunks;
  a.scale = 8.0 / r1 * std::sqrt(3.141592653589793 * t / (2.0 * s));
  a.partials = cv.take<double>((size_t)p.nchunks * r1 * q);
  double* Yd = cv.take<double>((size_t)r1 * q);
  const bool f64 = dt == FCT_F64;
  const bool overlap = p.nseg > 1 && c->fct2_overlap;
  hipStream_t side = c->stream;
  if (overlap) {
    int st = batch_ensure_aux(c, 0);
    if (st) return st;
    for (int k = 0; k < p.nseg; ++k)
      if (!c->ev_seg[k]) HIP_TRY(hipEventCreateWithFlags(&c->ev_seg[k], hipEventDisableTiming));
    side = c->branch[0];
    // three single-wave FJLT workgroups per CU keep HBM busy and leave the
    // rest of each CU to the contraction of the previous segment
    a.fjlt_grid = 3 * c->cus;
    // the side stream starts after everything queued so far (scratch reuse)
    HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
    HIP_TRY(hipStreamWaitEvent(side, c->ev_fork, 0));
  }
  // segment k: blocks [k bseg, (k + 1) bseg), columns [k bseg s, (k + 1) bseg s) of C
  int chunk0 = 0;
  prof_begin(c, 3);
  for (int k = 0; k < p.nseg; ++k) {
    a.beta0 = k * p.bseg;
    a.nbl = std::min(p.nb, (k + 1) * p.bseg) - a.beta0;
    HIP_TRY(launch_fct2_fjlt(a, f64, c->stream));
    if (!overlap) continue;
    HIP_TRY(hipEventRecord(c->ev_seg[k], c->stream));
    HIP_TRY(hipStreamWaitEvent(side, c->ev_seg[k], 0));
    if (k == 0) prof_begin(c, 4, side);
    a.mbase = a.beta0 * s;
    a.mend = std::min(p.K, (k + 1) * p.bseg * s);
    a.chunk0 = chunk0;
    a.nchunks = (int)((a.mend - a.mbase + p.kc - 1) / p.kc);
    chunk0 += a.nchunks;
    HIP_TRY(launch_fct2_cauchy(a, f64, side));
  }
  prof_end(c, 3);
  if (overlap) {
    prof_end(c, 4, side);
    HIP_TRY(hipEventRecord(c->ev_join[0], side));
    HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_join[0], 0));
  } else {
    prof_begin(c, 4);
    for (int k = 0; k < p.nseg; ++k) {
      a.mbase = k * p.bseg * s;
      a.mend = std::min(p.K, (k + 1) * p.bseg * s);
      a.chunk0 = chunk0;
      a.nchunks = (int)((a.mend - a.mbase + p.kc - 1) / p.kc);
      chunk0 += a.nchunks;
      HIP_TRY(launch_fct2_cauchy(a, f64, c->stream));
    }
    prof_end(c, 4);
  }
  HIP_TRY(launch_reduce_partials(a.partials, p.nchunks, r1, q, Y, Yd, c->flags + 0, true,
                                 c->stream, f64 ? 1 : 0));
  if (R) {
    double* work = cv.take<double>(qr_work_doubles(r1, q));
    HIP_TRY(launch_qr(Yd, r1, q, work, R, f64 ? 1e-13 : 1e-5, c->flags + 1, c->stream));
  }
  return FCT_OK;
}

int check_sketch_args(const fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda,
                      fct_dtype dt, const void* b, int32_t s, int32_t r1, bool want_r) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  const int q = d + (b ? 1 : 0);
  if (dt != FCT_F32 && dt != FCT_F64) return FCT_ERR_BAD_ARG;
  if (!is_pow2(s) || s < 2 || s > 4096) return FCT_ERR_BAD_ARG;
  if (r1 < q || r1 > 65536) return FCT_ERR_BAD_ARG;
  if (want_r && q > 88) return FCT_ERR_BAD_ARG;
  return FCT_OK;
}

struct ProbBufs {
  double* Md;
  float* Mf;
  float* Mfb;
  uint16_t* Mb;
  double* wg;
};

int run_probs(fct_ctx* c, Carve& cv, const void* X, const void* xb, int64_t n, int32_t d,
              int64_t lda, fct_dtype dt, const double* R, int32_t r2, uint64_t seed,
              float* lambda, double* sum_lambda, uint32_t flags, int32_t kb = 1,
              int64_t ldb = 0) {
  const int q = d + (xb ? kb : 0);
  const int r2p = r2_padded(r2);
  double* Md = cv.take<double>((size_t)q * r2p);
  float* Mf = cv.take<float>((size_t)q * r2p);
  float* Mfb = cv.take<float>((size_t)q * r2p);
  uint16_t* Mb = cv.take<uint16_t>((size_t)q * r2p);
  const int kind = dt == FCT_F64 ? kPass2F64 : (dt == FCT_BF16 ? kPass2BF16 : kPass2F32);
  const int grid = pass2_grid(n, kind, c->p2_wgs);
  double* wg = cv.take<double>((size_t)grid);
  HIP_TRY(launch_form_m(R, q, r2, r2p, seed, 0, Md, Mf, Mfb, Mb, c->flags + 1, c->stream,
                        (flags & FCT_FLAG_GAUSSIAN_PI2) != 0));
  Pass2Args a{};
  a.A = X;
  a.b = xb;
  a.lda = lda;
  a.ldb = ldb > 0 ? ldb : n;
  a.n = n;
  a.d = d;
  a.q = q;
  a.r2 = r2;
  a.M = dt == FCT_F64 ? (const void*)Md : (dt == FCT_BF16 ? (const void*)Mfb : (const void*)Mf);
  a.Mb = Mb;
  a.lambda = lambda;
  a.wg_sums = wg;
  prof_begin(c, 1);
  HIP_TRY(launch_pass2(a, kind, grid, c->stream));
  prof_end(c, 1);
  HIP_TRY(launch_sum_fixed(wg, grid, sum_lambda, c->stream));
  return FCT_OK;
}

template <typename C>
void carve_probs(C& cv, const fct_ctx* c, int q, int r2, int64_t n, int kind) {
  const int r2p = r2_padded(r2);
  cv.template take<double>((size_t)q * r2p);
  cv.template take<float>((size_t)q * r2p);
  cv.template take<float>((size_t)q * r2p);
  cv.template take<uint16_t>((size_t)q * r2p);
  cv.template take<double>((size_t)pass2_grid(n, kind, c->p2_wgs));
}

int run_select(fct_ctx* c, Carve& cv, const float* lambda, const double* sum_lambda, int64_t n,
               double s_out, uint64_t seed, int64_t cap, int64_t* idx, double* w, int64_t* S_dev,
               uint32_t instance = 0) {
  const int nb = select_grid(n);
  SelectArgs a{};
  a.lambda = lambda;
  a.sum_lambda = sum_lambda;
  a.n = n;
  a.s_out = s_out;
  a.seed = seed;
  a.instance = instance;
  a.p_out = nullptr;
  a.lookback = cv.take<uint64_t>((size_t)nb + 1);
  a.fail = c->flags + 1;
  a.idx = idx;
  a.w = w;
  a.cap = cap;
  a.S = S_dev;
  HIP_TRY(launch_select(a, c->stream));
  return FCT_OK;
}

template <typename C>
void carve_select(C& cv, int64_t n) {
  const int nb = select_grid(n);
  cv.template take<uint64_t>((size_t)nb + 1);
}

// The running-sum table of sampling with replacement.
struct RepCdf {
  double *bs, *pre, *cs, *co, *tot;
};
template <typename C>
void carve_rep(C& cv, int64_t n) {
  cv.template take<double>((size_t)rep_blocks(n));
  cv.template take<double>((size_t)rep_blocks(n));
  cv.template take<double>((size_t)rep_chunks(n));
  cv.template take<double>((size_t)rep_chunks(n));
  cv.template take<double>(1);
}
RepCdf take_rep(Carve& cv, int64_t n) {
  RepCdf r;
  r.bs = cv.take<double>((size_t)rep_blocks(n));
  r.pre = cv.take<double>((size_t)rep_blocks(n));
  r.cs = cv.take<double>((size_t)rep_chunks(n));
  r.co = cv.take<double>((size_t)rep_chunks(n));
  r.tot = cv.take<double>(1);
  return r;
}

}  // namespace

extern "C" {

int fct_create(fct_ctx** out, int device, void* hip_stream) {
  if (!out) return FCT_ERR_BAD_ARG;
  *out = nullptr;
  fct_ctx* c = new (std::nothrow) fct_ctx();
  if (!c) return FCT_ERR_OOM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return FCT_ERR_HIP;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return FCT_ERR_HIP;
    }
    c->own_stream = true;
  }
  if (device >= 0 && device < kNoAllocMaxDevices) {
    // once per device, with the device current: the address of its copy of
    // the static scratch (a failed lookup leaves only the no-allocation entry
    // point unusable)
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_noalloc_scratch)) == hipSuccess && ptr)
        g_noalloc_ptr[device] = ptr;
      else
        (void)hipGetLastError();
    }
    c->noalloc = g_noalloc_ptr[device];
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
    c->cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
      v > 0)
    c->lds_optin = (size_t)v;
  else if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
               hipSuccess && v > 0)
    c->lds_optin = (size_t)v;
  if (hipMalloc(&c->flags, 4 * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    fct_destroy(c);
    return FCT_ERR_OOM;
  }
  if (hipMemsetAsync(c->flags, 0, 4 * sizeof(int), c->stream) != hipSuccess) {
    fct_destroy(c);
    return FCT_ERR_HIP;
  }
  *out = c;
  return FCT_OK;
}

void fct_destroy(fct_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < fct_ctx::kProfKinds; ++k) {
    if (!c->prof_ev[k]) continue;
    for (int i = 0; i < 2 * fct_ctx::kProfSlots; ++i) (void)hipEventDestroy(c->prof_ev[k][i]);
    delete[] c->prof_ev[k];
  }
  if (c->bgraph) (void)hipGraphExecDestroy(c->bgraph);
  for (int k = 0; k < fct_ctx::kBranches; ++k) {
    if (c->branch[k]) (void)hipStreamDestroy(c->branch[k]);
    if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (int k = 0; k < fct_ctx::kFct2Segs; ++k)
    if (c->ev_seg[k]) (void)hipEventDestroy(c->ev_seg[k]);
  if (c->bpinned) (void)hipHostFree(c->bpinned);
  if (c->scratch) (void)hipFree(c->scratch);
  if (c->flags) (void)hipFree(c->flags);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* fct_strerror(int status) {
  switch (status) {
    case FCT_OK: return "ok";
    case FCT_ERR_BAD_ARG: return "bad argument";
    case FCT_ERR_OOM: return "out of device memory";
    case FCT_ERR_NONFINITE: return "non-finite value in input";
    case FCT_ERR_RANK_DEFICIENT: return "rank deficient";
    case FCT_ERR_HIP: return "HIP runtime error";
    case FCT_ERR_CAPACITY: return "coreset larger than capacity";
    default: return "unknown status";
  }
}

int fct_sync(fct_ctx* c) {
  if (!c) return FCT_ERR_BAD_ARG;
  return read_flags(c);
}

void* fct_stream(fct_ctx* c) { return c ? (void*)c->stream : nullptr; }

int fct_set_option(fct_ctx* c, int option, int64_t value) {
  if (!c) return FCT_ERR_BAD_ARG;
  switch (option) {
    case FCT_OPT_PASS1_KERNEL:
      if (value < FCT_P1_AUTO || value > FCT_P1_TILE) return FCT_ERR_BAD_ARG;
      c->p1_kernel = (int)value;
      return FCT_OK;
    case FCT_OPT_PASS1_WGS_PER_CU:
      if (value < 1 || value > 64) return FCT_ERR_BAD_ARG;
      c->p1_waves_of_wgs = (int)value;
      return FCT_OK;
    case FCT_OPT_PASS1_TILE_THREADS:
      if (value != 256 && value != 512 && value != 1024) return FCT_ERR_BAD_ARG;
      c->p1_threads = (int)value;
      return FCT_OK;
    case FCT_OPT_PASS2_WGS:
      if (value < 0 || value > (1 << 20)) return FCT_ERR_BAD_ARG;
      c->p2_wgs = (int)value;
      return FCT_OK;
    case FCT_OPT_SOLVE_WGS:
      if (value < 0 || value > 64) return FCT_ERR_BAD_ARG;
      c->irls_wgs = (int)value;
      return FCT_OK;
    case FCT_OPT_SOLVE_ROWS:
      if (value < 0 || value > (1 << 20)) return FCT_ERR_BAD_ARG;
      c->irls_rows = (int)value;
      return FCT_OK;
    case FCT_OPT_FCT2_OVERLAP:
      if (value != 0 && value != 1) return FCT_ERR_BAD_ARG;
      c->fct2_overlap = (int)value;
      return FCT_OK;
    default:
      return FCT_ERR_BAD_ARG;
  }
}

int fct_profile(fct_ctx* c, int enable) {
  if (!c) return FCT_ERR_BAD_ARG;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int k = 0; k < fct_ctx::kProfKinds; ++k) {
    c->prof_n[k] = 0;
    if (enable && !c->prof_ev[k]) {
      c->prof_ev[k] = new (std::nothrow) hipEvent_t[2 * fct_ctx::kProfSlots];
      if (!c->prof_ev[k]) return FCT_ERR_OOM;
      for (int i = 0; i < 2 * fct_ctx::kProfSlots; ++i)
        HIP_TRY(hipEventCreateWithFlags(&c->prof_ev[k][i], hipEventDefault));
    }
  }
  c->prof_on = enable != 0;
  return FCT_OK;
}

int fct_profile_read(fct_ctx* c, int kind, double* total_ms, int64_t* count) {
  if (!c || kind < 0 || kind >= fct_ctx::kProfKinds || !total_ms || !count) return FCT_ERR_BAD_ARG;
  HIP_TRY(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (int i = 0; i < c->prof_n[kind]; ++i) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, c->prof_ev[kind][2 * i], c->prof_ev[kind][2 * i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *count = c->prof_n[kind];
  return FCT_OK;
}

int fct_sketch(fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
               const void* b, int32_t s, int32_t r1, uint64_t seed, uint32_t flags, void* Y,
               double* R) {
  int st = check_sketch_args(c, A, n, d, lda, dt, b, s, r1, R != nullptr);
  if (st) return st;
  if (!Y && !R) return FCT_ERR_BAD_ARG;
  const int q = d + (b ? 1 : 0);
  const int64_t n_pad = (n + s - 1) / s * s;
  int perr = 0;
  const Pass1Plan p = make_pass1_plan(c, n_pad, q, s, r1, esize(dt), flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  Measure m;
  carve_sketch(m, p, n_pad, q, r1, esize(dt), R != nullptr);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  return run_sketch(c, cv, A, n, d, lda, dt, b, s, r1, seed, flags, Y, R, nullptr, p);
}

int fct_sketch_window(fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda,
                      fct_dtype dt, const void* b, int32_t s, int32_t r1, uint64_t seed,
                      int64_t row0, uint32_t flags, void* Y) {
  int st = check_sketch_args(c, A, n, d, lda, dt, b, s, r1, false);
  if (st) return st;
  if (!Y || row0 < 0 || row0 % s != 0 || row0 % 256 != 0) return FCT_ERR_BAD_ARG;
  const int q = d + (b ? 1 : 0);
  const int64_t n_pad = (n + s - 1) / s * s;
  int perr = 0;
  const Pass1Plan p = make_pass1_plan(c, n_pad, q, s, r1, esize(dt), flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  Measure m;
  carve_sketch(m, p, n_pad, q, r1, esize(dt), false);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  return run_sketch(c, cv, A, n, d, lda, dt, b, s, r1, seed, flags, Y, nullptr, nullptr, p, row0);
}

int fct2_sketch(fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
                const void* b, int32_t t, int32_t s, int32_t r1, uint64_t seed, void* Y,
                double* R) {
  int st = check_fct2_args(c, A, n, d, lda, dt, b, t, s, r1, R != nullptr);
  if (st) return st;
  if (!Y && !R) return FCT_ERR_BAD_ARG;
  const int q = d + (b ? 1 : 0);
  const Fct2Plan p = make_fct2_plan(n, q, t, s, r1, c->fct2_overlap != 0);
  Measure m;
  carve_fct2(m, p, q, r1, R != nullptr);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  return run_fct2(c, cv, A, n, d, lda, dt, b, t, s, r1, seed, Y, R, p);
}

int l1_sample_probs_ex(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d,
                       int64_t lda, fct_dtype dt, const double* R, int32_t r2, uint64_t seed,
                       int64_t s_out, uint32_t flags, float* lambda, float* p, double* sum_lambda) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (dt != FCT_F32 && dt != FCT_F64 && dt != FCT_BF16) return FCT_ERR_BAD_ARG;
  if (!R || r2 < 1 || r2 > 32 || s_out < 1) return FCT_ERR_BAD_ARG;
  const int q = d + (b ? 1 : 0);
  const int kind = dt == FCT_F64 ? kPass2F64 : (dt == FCT_BF16 ? kPass2BF16 : kPass2F32);
  Measure m;
  if (!lambda) m.take<float>((size_t)n);
  if (!sum_lambda) m.take<double>(1);
  carve_probs(m, c, q, r2, n, kind);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  float* lam = lambda ? lambda : cv.take<float>((size_t)n);
  double* sl = sum_lambda ? sum_lambda : cv.take<double>(1);
  if ((st = run_probs(c, cv, A, b, n, d, lda, dt, R, r2, seed, lam, sl, flags))) return st;
  if (p) {
    SelectArgs a{};
    a.lambda = lam;
    a.sum_lambda = sl;
    a.n = n;
    a.s_out = (double)s_out;
    a.p_out = p;
    HIP_TRY(launch_probs_only(a, c->stream));
  }
  return FCT_OK;
}

int l1_sample_probs_noalloc(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d,
                            int64_t lda, fct_dtype dt, const double* R, int32_t r2, uint64_t seed,
                            int64_t s_out, uint32_t flags, float* lambda, float* p,
                            double* sum_lambda) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (dt != FCT_F32 && dt != FCT_F64 && dt != FCT_BF16) return FCT_ERR_BAD_ARG;
  if (!R || r2 < 1 || r2 > 32 || s_out < 1 || !lambda || !sum_lambda) return FCT_ERR_BAD_ARG;
  const int q = d + (b ? 1 : 0);
  if (q > (dt == FCT_F64 ? 96 : 65)) return FCT_ERR_BAD_ARG;
  if (!c->noalloc) return FCT_ERR_HIP;
  const int kind = dt == FCT_F64 ? kPass2F64 : (dt == FCT_BF16 ? kPass2BF16 : kPass2F32);
  Measure m;
  carve_probs(m, c, q, r2, n, kind);
  if (m.off > kNoAllocBytes) return FCT_ERR_CAPACITY;  // a pass-2 grid above the scratch
  Carve cv(reinterpret_cast<char*>(c->noalloc));
  if ((st = run_probs(c, cv, A, b, n, d, lda, dt, R, r2, seed, lambda, sum_lambda, flags)))
    return st;
  if (p) {
    SelectArgs a{};
    a.lambda = lambda;
    a.sum_lambda = sum_lambda;
    a.n = n;
    a.s_out = (double)s_out;
    a.p_out = p;
    HIP_TRY(launch_probs_only(a, c->stream));
  }
  return FCT_OK;
}

int l1_sample_probs(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
                    fct_dtype dt, const double* R, int32_t r2, uint64_t seed, int64_t s_out,
                    float* lambda, float* p, double* sum_lambda) {
  return l1_sample_probs_ex(c, A, b, n, d, lda, dt, R, r2, seed, s_out, 0u, lambda, p,
                            sum_lambda);
}

// Optional copies of an instance's intermediate results (batched form).
struct CoresetOut {
  double* R = nullptr;
  float* lambda = nullptr;
  int64_t* idx = nullptr;
  int64_t idx_cap = 0;
};

static int coreset_impl(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d,
                        int64_t lda, fct_dtype dt, const void* A_lowp, const void* b_lowp,
                        int64_t ld_lowp, const fct_params* prm, int64_t cap, void* At, void* bt,
                        double* w, int64_t* idx, int64_t* S_dev, Carve& cv,
                        const CoresetOut* out = nullptr) {
  const int q = d + 1;
  const bool fct2 = (prm->flags & FCT_FLAG_FCT2) != 0;
  const int64_t n_pad = (n + prm->s - 1) / prm->s * prm->s;
  int perr = 0;
  const Pass1Plan p =
      fct2 ? Pass1Plan{} : make_pass1_plan(c, n_pad, q, prm->s, prm->r1, esize(dt), prm->flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  double* R = cv.take<double>((size_t)q * q);
  float* lam = cv.take<float>((size_t)n);
  double* sl = cv.take<double>(1);
  int st;
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if (fct2)
      st = run_fct2(c, sub, A, n, d, lda, dt, b, prm->s, prm->s2, prm->r1, prm->seed, nullptr, R,
                    make_fct2_plan(n, q, prm->s, prm->s2, prm->r1, c->fct2_overlap != 0));
    else
      st = run_sketch(c, sub, A, n, d, lda, dt, b, prm->s, prm->r1, prm->seed, prm->flags,
                      nullptr, R, nullptr, p);
    if (st) return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    const bool lowp = A_lowp != nullptr;
    if ((st = run_probs(c, sub, lowp ? A_lowp : A, lowp ? b_lowp : b, n, d, lowp ? ld_lowp : lda,
                        lowp ? FCT_BF16 : dt, R, prm->r2, prm->seed, lam, sl, prm->flags)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_select(c, sub, lam, sl, n, (double)prm->s_out, prm->seed, cap, idx, w, S_dev)))
      return st;
  }
  HIP_TRY(launch_gather(A, b, lda, d, 1, n, idx, S_dev, cap, At, bt, cap, dt == FCT_F64, c->stream));
  if (out && out->R)
    HIP_TRY(hipMemcpyAsync(out->R, R, (size_t)q * q * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  if (out && out->lambda)
    HIP_TRY(hipMemcpyAsync(out->lambda, lam, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice,
                           c->stream));
  if (out && out->idx && out->idx_cap > 0)
    HIP_TRY(hipMemcpyAsync(out->idx, idx, (size_t)std::min(cap, out->idx_cap) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, c->stream));
  return FCT_OK;
}

static size_t coreset_scratch(const fct_ctx* c, int64_t n, int32_t d, fct_dtype dt,
                              const fct_params* prm, bool lowp) {
  const int q = d + 1;
  const bool fct2 = (prm->flags & FCT_FLAG_FCT2) != 0;
  const int64_t n_pad = (n + prm->s - 1) / prm->s * prm->s;
  int perr = 0;
  Measure m;
  m.take<double>((size_t)q * q);
  m.take<float>((size_t)n);
  m.take<double>(1);
  const size_t base = m.off;
  Measure a, bb, cc;
  if (fct2) {
    carve_fct2(a, make_fct2_plan(n, q, prm->s, prm->s2, prm->r1, c->fct2_overlap != 0), q,
               prm->r1, true);
  } else {
    const Pass1Plan p =
        make_pass1_plan(c, n_pad, q, prm->s, prm->r1, esize(dt), prm->flags, &perr);
    carve_sketch(a, p, n_pad, q, prm->r1, esize(dt), true);
  }
  carve_probs(bb, c, q, prm->r2, n, lowp ? kPass2BF16 : (dt == FCT_F64 ? kPass2F64 : kPass2F32));
  carve_select(cc, n);
  size_t mx = a.off;
  if (bb.off > mx) mx = bb.off;
  if (cc.off > mx) mx = cc.off;
  return base + mx + 1024;
}

// FCT_FLAG_FCT2 is taken by l1_regress and l1_coreset only (allow_fct2).
static int check_params(const fct_params* prm, int q, bool allow_fct2 = false) {
  if (!prm) return FCT_ERR_BAD_ARG;
  if (!is_pow2(prm->s) || prm->s < 2 || prm->s > 4096) return FCT_ERR_BAD_ARG;
  if (prm->flags & FCT_FLAG_FCT2) {
    if (!allow_fct2 || prm->s < 64 || prm->s2 < 1 || prm->s2 > prm->s || prm->s2 > kFct2MaxS)
      return FCT_ERR_BAD_ARG;
  }
  if (prm->r1 < q || prm->r1 > 65536 || prm->r2 < 1 || prm->r2 > 32) return FCT_ERR_BAD_ARG;
  if (q > 65) return FCT_ERR_BAD_ARG;  // solver and panel QR limits: d <= 64
  return FCT_OK;
}

int l1_coreset(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
               fct_dtype dt, const void* A_lowp, const void* b_lowp, int64_t ld_lowp,
               const fct_params* prm, int64_t cap, void* At, void* bt, double* w, int64_t* idx,
               int64_t* S) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!b || (dt != FCT_F32 && dt != FCT_F64)) return FCT_ERR_BAD_ARG;
  if ((st = check_params(prm, d + 1, true))) return st;
  if (prm->s_out < 1 || cap < 1 || !At || !bt || !w || !idx || !S) return FCT_ERR_BAD_ARG;
  if (A_lowp && (!b_lowp || ld_lowp < n)) return FCT_ERR_BAD_ARG;
  const size_t need = coreset_scratch(c, n, d, dt, prm, A_lowp != nullptr) + 256;
  if ((st = ensure_scratch(c, need))) return st;
  Carve cv(c->scratch);
  int64_t* S_dev = cv.take<int64_t>(1);
  if ((st = coreset_impl(c, A, b, n, d, lda, dt, A_lowp, b_lowp, ld_lowp, prm, cap, At, bt, w,
                         idx, S_dev, cv)))
    return st;
  HIP_TRY(hipMemcpyAsync(c->pinned, S_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);  // synchronizes
  std::memcpy(S, c->pinned, sizeof(int64_t));
  if (fl) return fl;
  if (*S > cap) return FCT_ERR_CAPACITY;
  return FCT_OK;
}

int l1_select(fct_ctx* c, const float* lambda, const double* sum_lambda, int64_t n, int64_t s_out,
              uint64_t seed, int64_t cap, int64_t* idx, double* w, int64_t* S) {
  if (!c || !lambda || !sum_lambda || n < 1 || s_out < 1 || cap < 1 || !idx || !w || !S)
    return FCT_ERR_BAD_ARG;
  Measure m;
  m.take<int64_t>(1);
  carve_select(m, n);
  int st;
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  int64_t* S_dev = cv.take<int64_t>(1);
  if ((st = run_select(c, cv, lambda, sum_lambda, n, (double)s_out, seed, cap, idx, w, S_dev)))
    return st;
  HIP_TRY(hipMemcpyAsync(c->pinned, S_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);
  std::memcpy(S, c->pinned, sizeof(int64_t));
  if (fl) return fl;
  return *S > cap ? FCT_ERR_CAPACITY : FCT_OK;
}

int l1_select_draw(fct_ctx* c, const float* lambda, const double* sum_lambda, int64_t n,
                   int64_t s_out, uint64_t seed, int32_t draw, int32_t mode, int64_t cap,
                   int64_t* idx, double* w, int64_t* S) {
  if (!c || !lambda || n < 1 || s_out < 1 || cap < 1 || !idx || !w || !S || draw < 0)
    return FCT_ERR_BAD_ARG;
  if (mode == FCT_SAMPLE_BERNOULLI && !sum_lambda) return FCT_ERR_BAD_ARG;
  if (mode != FCT_SAMPLE_BERNOULLI && mode != FCT_SAMPLE_REPLACE) return FCT_ERR_BAD_ARG;
  if (mode == FCT_SAMPLE_REPLACE && cap < s_out) return FCT_ERR_BAD_ARG;
  Measure m;
  m.take<int64_t>(1);
  if (mode == FCT_SAMPLE_BERNOULLI) carve_select(m, n);
  else carve_rep(m, n);
  int st;
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  int64_t* S_dev = cv.take<int64_t>(1);
  if (mode == FCT_SAMPLE_BERNOULLI) {
    if ((st = run_select(c, cv, lambda, sum_lambda, n, (double)s_out, seed, cap, idx, w, S_dev,
                         (uint32_t)draw)))
      return st;
  } else {
    const RepCdf r = take_rep(cv, n);
    HIP_TRY(launch_select_replace(lambda, n, s_out, seed, (uint32_t)draw, r.bs, r.pre, r.cs, r.co,
                                  r.tot, true, idx, w, S_dev, c->stream));
  }
  HIP_TRY(hipMemcpyAsync(c->pinned, S_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);
  std::memcpy(S, c->pinned, sizeof(int64_t));
  if (fl) return fl;
  return *S > cap ? FCT_ERR_CAPACITY : FCT_OK;
}

int l1_solve(fct_ctx* c, const void* At, const void* bt, const double* w, int64_t S, int32_t d,
             int64_t ldat, fct_dtype dt, int32_t iters, double* x, double* obj) {
  if (!c || !At || !bt || !w || S < 1 || d < 1 || d > 64 || ldat < S || !x) return FCT_ERR_BAD_ARG;
  if (dt != FCT_F32 && dt != FCT_F64) return FCT_ERR_BAD_ARG;
  if (iters <= 0) iters = 80;
  Measure m;
  m.take<int64_t>(1);
  m.take<double>(irls_work_doubles(S, d));
  m.take<double>(128);
  int st;
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  int64_t* S_dev = cv.take<int64_t>(1);
  double* work = cv.take<double>(irls_work_doubles(S, d));
  double* outv = cv.take<double>(128);
  std::memcpy((char*)c->pinned + 2048, &S, sizeof(int64_t));
  HIP_TRY(hipMemcpyAsync(S_dev, (char*)c->pinned + 2048, sizeof(int64_t), hipMemcpyHostToDevice,
                         c->stream));
  prof_begin(c, 2);
  HIP_TRY(launch_irls(At, bt, w, S_dev, S, S, d, ldat, dt == FCT_F64, iters, work, outv,
                      outv + 64, c->flags + 1, c->stream, c->irls_rows, c->irls_wgs));
  prof_end(c, 2);
  HIP_TRY(hipMemcpyAsync(c->pinned, outv, 65 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);
  const double* h = reinterpret_cast<const double*>(c->pinned);
  for (int i = 0; i < d; ++i) x[i] = h[i];
  if (obj) *obj = h[64];
  return fl;
}

int l1_regress(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
               fct_dtype dt, const void* A_lowp, const void* b_lowp, int64_t ld_lowp, double eps,
               const fct_params* prm_in, double* x, double* obj, int64_t* S_out) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!b || !x || !prm_in || (dt != FCT_F32 && dt != FCT_F64)) return FCT_ERR_BAD_ARG;
  fct_params prm = *prm_in;
  if (prm.s_out <= 0) {
    if (!(eps > 0.0)) return FCT_ERR_BAD_ARG;
    prm.s_out = (int64_t)std::ceil(20.0 * (d + 1) / eps);
  }
  if ((st = check_params(&prm, d + 1, true))) return st;
  if (A_lowp && (!b_lowp || ld_lowp < n)) return FCT_ERR_BAD_ARG;
  const int iters = prm.irls_iters > 0 ? prm.irls_iters : 80;
  int64_t cap = 2 * prm.s_out + 8 * (int64_t)std::sqrt((double)prm.s_out) + 1024;
  if (cap > n) cap = n;
  const size_t es = esize(dt);
  for (int attempt = 0; attempt < 2; ++attempt) {
    Measure m;
    m.take<int64_t>(1);
    m.take<char>((size_t)cap * d * es);
    m.take<char>((size_t)cap * es);
    m.take<double>((size_t)cap);
    m.take<int64_t>((size_t)cap);
    m.take<double>(irls_work_doubles(cap, d));
    m.take<double>(128);
    const size_t need = m.off + coreset_scratch(c, n, d, dt, &prm, A_lowp != nullptr) + 256;
    if ((st = ensure_scratch(c, need))) return st;
    Carve cv(c->scratch);
    int64_t* S_dev = cv.take<int64_t>(1);
    char* At = cv.take<char>((size_t)cap * d * es);
    char* bt = cv.take<char>((size_t)cap * es);
    double* w = cv.take<double>((size_t)cap);
    int64_t* idx = cv.take<int64_t>((size_t)cap);
    double* work = cv.take<double>(irls_work_doubles(cap, d));
    double* outv = cv.take<double>(128);
    Carve rest(c->scratch);
    rest.off = cv.off;
    if ((st = coreset_impl(c, A, b, n, d, lda, dt, A_lowp, b_lowp, ld_lowp, &prm, cap, At, bt, w,
                           idx, S_dev, rest)))
      return st;
    prof_begin(c, 2);
    const int64_t S_hint = prm.s_out < cap ? prm.s_out : cap;
    HIP_TRY(launch_irls(At, bt, w, S_dev, cap, S_hint, d, cap, dt == FCT_F64, iters, work, outv,
                        outv + 64, c->flags + 1, c->stream, c->irls_rows, c->irls_wgs));
    prof_end(c, 2);
    HIP_TRY(hipMemcpyAsync(c->pinned, outv, 65 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync((char*)c->pinned + 1024, S_dev, sizeof(int64_t), hipMemcpyDeviceToHost,
                           c->stream));
    const int fl = read_flags(c);
    int64_t S;
    std::memcpy(&S, (char*)c->pinned + 1024, sizeof(int64_t));
    if (S_out) *S_out = S;
    if (fl) return fl;
    if (S > cap) {
      cap = S + S / 8 + 1024;
      continue;
    }
    const double* h = reinterpret_cast<const double*>(c->pinned);
    for (int i = 0; i < d; ++i) x[i] = h[i];
    if (obj) *obj = h[64];
    return FCT_OK;
  }
  return FCT_ERR_CAPACITY;
}


// ---- batched form ----------------------------------------------------------

namespace {

__global__ void batch_collect_kernel(const IrlsArgs* __restrict__ arr, int count,
                                     double* __restrict__ out) {
  // out row i: [0, 64) x, [64] objective, [65] S, [66] solver status
  const int i = blockIdx.x;
  if (i >= count) return;
  const IrlsArgs a = arr[i];
  for (int k = threadIdx.x; k < a.d; k += blockDim.x) out[i * 72 + k] = a.x_out[k];
  if (threadIdx.x == 0) {
    out[i * 72 + 64] = *a.obj_out;
    out[i * 72 + 65] = (double)*a.S_dev;
    out[i * 72 + 66] = (double)*a.status;
  }
}

struct BatchItem {
  fct_params prm;
  int64_t cap;
  size_t off;     // byte offset of the instance's region in the scratch arena
  size_t bytes;
  int nwg = 1;    // workgroups of the instance's solve
};

// Block maps of the batched solve: the instances with several workgroups
// (one launch, big.size() blocks), then the rest (one block each).
struct BatchSolvePlan {
  std::vector<int> big, small;
};

// The FCT1 block size of the paper's experiments (section "Numerical
// experiments"): ceil(2 d ln d), here rounded up to a power of two within
// [64, 1024] (the butterflies work on powers of two; 64 keeps the blocks of
// small d at the width of a wave).
int batch_block_size(int d) {
  const double t = std::ceil(2.0 * d * std::log((double)d));
  int s = 64;
  while (s < t && s < 1024) s <<= 1;
  return s;
}

int batch_ensure_aux(fct_ctx* c, size_t pinned_bytes) {
  if (!c->branch[0]) {
    for (int k = 0; k < fct_ctx::kBranches; ++k) {
      HIP_TRY(hipStreamCreateWithFlags(&c->branch[k], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  }
  if (c->bpinned_bytes < pinned_bytes) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->bpinned) HIP_TRY(hipHostFree(c->bpinned));
    c->bpinned = nullptr;
    c->bpinned_bytes = 0;
    HIP_TRY(hipHostMalloc(&c->bpinned, pinned_bytes, hipHostMallocDefault));
    c->bpinned_bytes = pinned_bytes;
  }
  return FCT_OK;
}

// Every instance's steps 1-7 on the forked streams, then the batched solve
// and the collection of outputs on the context stream.
int batch_enqueue(fct_ctx* c, const fct_instance* inst, int count, fct_dtype dt,
                  const std::vector<BatchItem>& items, const IrlsArgs* args_dev, double* out_dev,
                  size_t out_bytes, const BatchSolvePlan& sp, const int* map_dev) {
  const size_t es = esize(dt);
  HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
  for (int k = 0; k < fct_ctx::kBranches; ++k) HIP_TRY(hipStreamWaitEvent(c->branch[k], c->ev_fork, 0));
  hipStream_t main = c->stream;
  int st = FCT_OK;
  for (int i = 0; i < count && st == FCT_OK; ++i) {
    const fct_instance& in = inst[i];
    const BatchItem& it = items[i];
    const int d = in.d;
    Carve cv(c->scratch);
    cv.off = it.off;
    int64_t* S_dev = cv.take<int64_t>(1);
    char* At = cv.take<char>((size_t)it.cap * d * es);
    char* bt = cv.take<char>((size_t)it.cap * es);
    double* w = cv.take<double>((size_t)it.cap);
    int64_t* idx = cv.take<int64_t>((size_t)it.cap);
    cv.take<double>(irls_batched_work_doubles(d, it.nwg));
    cv.take<double>(72);
    cv.take<int>(4);
    Carve rest(c->scratch);
    rest.off = cv.off;
    c->stream = c->branch[i % fct_ctx::kBranches];
    CoresetOut out;
    out.R = in.R_out;
    out.lambda = in.lambda_out;
    out.idx = in.idx_out;
    out.idx_cap = in.idx_cap;
    st = coreset_impl(c, in.A, in.b, in.n, d, in.lda, dt, in.A_lowp, in.b_lowp, in.ld_lowp, &it.prm,
                      it.cap, At, bt, w, idx, S_dev, rest, &out);
    c->stream = main;
  }
  if (st) return st;
  for (int k = 0; k < fct_ctx::kBranches; ++k) {
    HIP_TRY(hipEventRecord(c->ev_join[k], c->branch[k]));
    HIP_TRY(hipStreamWaitEvent(main, c->ev_join[k], 0));
  }
  if (sp.big.empty()) {
    HIP_TRY(launch_irls_batched(args_dev, count, dt == FCT_F64, main));
  } else {
    HIP_TRY(launch_irls_batched(args_dev, count, dt == FCT_F64, main, map_dev, (int)sp.big.size(), true));
    if (!sp.small.empty())
      HIP_TRY(launch_irls_batched(args_dev, count, dt == FCT_F64, main, map_dev + sp.big.size(),
                                  (int)sp.small.size(), false));
  }
  hipLaunchKernelGGL(batch_collect_kernel, dim3(count), dim3(64), 0, main, args_dev, count, out_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->bpinned, out_dev, out_bytes, hipMemcpyDeviceToHost, main));
  return FCT_OK;
}

}  // namespace

int l1_regress_batched(fct_ctx* c, const fct_instance* inst, int32_t count, fct_dtype dt,
                       double eps, double* x, double* obj, int64_t* S, int32_t* s_used,
                       int32_t* status) {
  if (!c || !inst || count < 1 || !x || !status) return FCT_ERR_BAD_ARG;
  if (dt != FCT_F32 && dt != FCT_F64) return FCT_ERR_BAD_ARG;
  struct ProfOff {  // no timing events inside a batch (they would be captured)
    fct_ctx* c;
    bool saved;
    explicit ProfOff(fct_ctx* cc) : c(cc), saved(cc->prof_on) { c->prof_on = false; }
    ~ProfOff() { c->prof_on = saved; }
  } prof_off(c);
  int st;
  std::vector<BatchItem> items((size_t)count);
  const size_t es = esize(dt);
  // arguments, block sizes, sizes
  for (int i = 0; i < count; ++i) {
    const fct_instance& in = inst[i];
    if ((st = check_common(c, in.A, in.n, in.d, in.lda))) return st;
    if (!in.b || in.d > 64) return FCT_ERR_BAD_ARG;
    if (in.A_lowp && (!in.b_lowp || in.ld_lowp < in.n || dt != FCT_F32)) return FCT_ERR_BAD_ARG;
    fct_params prm = in.prm;
    if (prm.s_out <= 0) {
      if (!(eps > 0.0)) return FCT_ERR_BAD_ARG;
      prm.s_out = (int64_t)std::ceil(20.0 * (in.d + 1) / eps);
    }
    if (prm.irls_iters <= 0) prm.irls_iters = 80;
    items[i].prm = prm;
  }
  for (int i = 0; i < count; ++i) {
    fct_params& prm = items[i].prm;
    if (prm.s == 0) prm.s = batch_block_size(inst[i].d);
  }
  for (int i = 0; i < count; ++i) {
    fct_params& prm = items[i].prm;
    if ((st = check_params(&prm, inst[i].d + 1))) return st;
    int64_t cap = 2 * prm.s_out + 8 * (int64_t)std::sqrt((double)prm.s_out) + 1024;
    if (cap > inst[i].n) cap = inst[i].n;
    items[i].cap = cap;
  }
  // The solve of an instance costs about cap (d + 1)^2 per reweighting.  One
  // workgroup holds a whole CU (its LDS), so with one each the largest
  // instances finish long after the rest.  The instances within 4x of the
  // largest cost get several workgroups each (as many as the device holds at
  // once, shared out, at most one per 256 coreset rows) in a launch of their
  // own; the rest follow, one workgroup each.
  BatchSolvePlan sp;
  {
    std::vector<double> cost((size_t)count);
    double mx = 0.0;
    for (int i = 0; i < count; ++i) {
      cost[i] = (double)items[i].cap * (inst[i].d + 1) * (inst[i].d + 1);
      mx = std::max(mx, cost[i]);
    }
    int nbig = 0;
    for (int i = 0; i < count; ++i) nbig += cost[i] * 4.0 >= mx;
    const int resident = irls_max_resident_wgs(c->cus);
    const int per = nbig > 0 ? resident / nbig : 0;
    if (per >= 2) {
      for (int i = 0; i < count; ++i) {
        if (cost[i] * 4.0 >= mx) {
          const int byrows = (int)std::max<int64_t>(1, items[i].cap / 256);
          items[i].nwg = std::min(std::min(per, byrows), 64);
          for (int k = 0; k < items[i].nwg; ++k) sp.big.push_back(i);
        } else {
          sp.small.push_back(i);
        }
      }
      if (sp.big.empty()) sp.small.clear();
    }
  }
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    fct_params& prm = items[i].prm;
    const int d = inst[i].d;
    const int64_t cap = items[i].cap;
    Measure m;
    m.take<int64_t>(1);
    m.take<char>((size_t)cap * d * es);
    m.take<char>((size_t)cap * es);
    m.take<double>((size_t)cap);
    m.take<int64_t>((size_t)cap);
    m.take<double>(irls_batched_work_doubles(d, items[i].nwg));
    m.take<double>(72);
    m.take<int>(4);
    const size_t bytes = m.off + coreset_scratch(c, inst[i].n, d, dt, &prm, inst[i].A_lowp != nullptr) + 512;
    items[i].off = total;
    items[i].bytes = bytes;
    total += (bytes + 255) & ~size_t(255);
  }
  const size_t args_off = total;
  const size_t map_count = sp.big.size() + sp.small.size();
  const size_t args_bytes = (size_t)count * sizeof(IrlsArgs) + map_count * sizeof(int);
  total += (args_bytes + 255) & ~size_t(255);
  const size_t out_off = total;
  const size_t out_bytes = (size_t)count * 72 * sizeof(double);
  total += out_bytes + 256;
  if ((st = ensure_scratch(c, total))) return st;
  const size_t pin_bytes = args_bytes > out_bytes ? args_bytes : out_bytes;
  if ((st = batch_ensure_aux(c, pin_bytes))) return st;
  IrlsArgs* args_dev = reinterpret_cast<IrlsArgs*>(c->scratch + args_off);
  int* map_dev = reinterpret_cast<int*>(c->scratch + args_off + (size_t)count * sizeof(IrlsArgs));
  double* out_dev = reinterpret_cast<double*>(c->scratch + out_off);
  // per-instance solver arguments (pointers into each instance's region)
  std::vector<IrlsArgs> args((size_t)count);
  for (int i = 0; i < count; ++i) {
    const int d = inst[i].d;
    Carve cv(c->scratch);
    cv.off = items[i].off;
    IrlsArgs& a = args[i];
    a.S_dev = cv.take<int64_t>(1);
    a.At = cv.take<char>((size_t)items[i].cap * d * es);
    a.bt = cv.take<char>((size_t)items[i].cap * es);
    a.w = cv.take<double>((size_t)items[i].cap);
    cv.take<int64_t>((size_t)items[i].cap);
    const int nwg = items[i].nwg;
    double* work = cv.take<double>(irls_batched_work_doubles(d, nwg));
    double* outv = cv.take<double>(72);
    a.status = cv.take<int>(4);
    a.cap = items[i].cap;
    a.ldat = items[i].cap;
    a.d = d;
    a.iters = items[i].prm.irls_iters;
    // one workgroup takes every row; several share them about evenly
    a.row_target = nwg > 1 ? (int)((items[i].cap + nwg - 1) / nwg) : 1 << 30;
    a.part = work;
    a.bar = irls_batched_bar(work, d, nwg);
    a.x_out = outv;
    a.obj_out = outv + 64;
    a.wg0 = 0;
    a.nwg = nwg;
  }
  // block maps: each big instance's first block, then the small ones in turn
  std::vector<int> map;
  map.reserve(map_count);
  for (size_t b = 0; b < sp.big.size(); ++b) {
    const int i = sp.big[b];
    if (b == 0 || sp.big[b - 1] != i) args[i].wg0 = (int)b;
    map.push_back(i);
  }
  for (size_t b = 0; b < sp.small.size(); ++b) {
    args[sp.small[b]].wg0 = (int)b;
    map.push_back(sp.small[b]);
  }
  // signature of this batch: instances, parameters, arena
  std::vector<char> sig;
  auto put = [&sig](const void* p, size_t nb) {
    const char* q = reinterpret_cast<const char*>(p);
    sig.insert(sig.end(), q, q + nb);
  };
  put(&count, sizeof(count));
  put(&dt, sizeof(dt));
  put(&c->scratch, sizeof(c->scratch));
  put(&c->scratch_bytes, sizeof(c->scratch_bytes));
  put(&c->stream, sizeof(c->stream));
  for (int i = 0; i < count; ++i) {
    put(&inst[i], sizeof(fct_instance));
    put(&items[i].prm, sizeof(fct_params));
  }
  const bool replay = c->bgraph && sig == c->bsig;
  if (!replay) {
    std::memcpy(c->bpinned, args.data(), (size_t)count * sizeof(IrlsArgs));
    if (!map.empty())
      std::memcpy((char*)c->bpinned + (size_t)count * sizeof(IrlsArgs), map.data(), map.size() * sizeof(int));
    HIP_TRY(hipMemcpyAsync(args_dev, c->bpinned, args_bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->bgraph) {
      (void)hipGraphExecDestroy(c->bgraph);
      c->bgraph = nullptr;
      c->bsig.clear();
    }
    // capture; if the runtime refuses, run the same sequence eagerly
    bool captured = false;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
      const int est = batch_enqueue(c, inst, count, dt, items, args_dev, out_dev, out_bytes, sp, map_dev);
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(c->stream, &g);
      if (est == FCT_OK && ee == hipSuccess && g) {
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
          c->bgraph = ex;
          c->bsig = sig;
          captured = true;
        }
      }
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
    }
    if (captured) {
      HIP_TRY(hipGraphLaunch(c->bgraph, c->stream));
    } else {
      if ((st = batch_enqueue(c, inst, count, dt, items, args_dev, out_dev, out_bytes, sp, map_dev)))
        return st;
    }
  } else {
    HIP_TRY(hipGraphLaunch(c->bgraph, c->stream));
  }
  const int fl = read_flags(c);  // waits for the batch
  const double* h = reinterpret_cast<const double*>(c->bpinned);
  int first = FCT_OK;
  int64_t off = 0;
  for (int i = 0; i < count; ++i) {
    const int d = inst[i].d;
    const double* row = h + (size_t)i * 72;
    const int64_t Si = (int64_t)row[65];
    int sti = (int)row[66];
    if (Si > items[i].cap) sti = FCT_ERR_CAPACITY;
    status[i] = sti;
    for (int k = 0; k < d; ++k) x[off + k] = row[k];
    off += d;
    if (obj) obj[i] = row[64];
    if (S) S[i] = Si;
    if (s_used) s_used[i] = items[i].prm.s;
    if (sti != FCT_OK && first == FCT_OK) first = sti;
  }
  if (fl) return fl;
  return first;
}

// Workgroups per instance of a batched solve over `count` alike instances
// of at most cap coreset rows: the workgroups the device holds at once,
// shared out, at most one per 256 rows and 64 (1: one workgroup each).
static int alike_solve_wgs(const fct_ctx* c, int count, int64_t cap) {
  const int resident = irls_max_resident_wgs(c->cus);
  int64_t w = count > 0 ? resident / count : 1;
  w = std::min<int64_t>(w, std::max<int64_t>(1, cap / 256));
  w = std::min<int64_t>(w, 64);
  return (int)std::max<int64_t>(w, 1);
}

// bytes of `count` solver arguments followed by their block map
static size_t solve_args_bytes(int count, int nwg) {
  return (size_t)count * sizeof(IrlsArgs) + (nwg > 1 ? (size_t)count * nwg * sizeof(int) : 0);
}

// coreset rows per workgroup: all of them for one, an even share for several
static int solve_row_target(int64_t cap, int nwg) {
  return nwg > 1 ? (int)((cap + nwg - 1) / nwg) : 1 << 30;
}

// Instance k's blocks are k nwg .. k nwg + nwg - 1: its first block, the
// block map after the arguments, both copied to the device (through the
// pinned block, which the caller then waits for).
static int upload_solve_args(fct_ctx* c, std::vector<IrlsArgs>& args, int nwg, IrlsArgs* args_dev) {
  const int count = (int)args.size();
  for (int k = 0; k < count; ++k) {
    args[k].wg0 = k * nwg;
    args[k].nwg = nwg;
  }
  std::memcpy(c->bpinned, args.data(), (size_t)count * sizeof(IrlsArgs));
  if (nwg > 1) {
    int* map = reinterpret_cast<int*>((char*)c->bpinned + (size_t)count * sizeof(IrlsArgs));
    for (int b = 0; b < count * nwg; ++b) map[b] = b / nwg;
  }
  HIP_TRY(hipMemcpyAsync(args_dev, c->bpinned, solve_args_bytes(count, nwg), hipMemcpyHostToDevice,
                         c->stream));
  return FCT_OK;
}

static hipError_t launch_solve_alike(const IrlsArgs* args_dev, int count, bool f64, hipStream_t st, int nwg) {
  if (nwg <= 1) return launch_irls_batched(args_dev, count, f64, st);
  const int* map = reinterpret_cast<const int*>(args_dev + count);
  return launch_irls_batched(args_dev, count, f64, st, map, count * nwg, true);
}

int l1_regress_multi(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
                     fct_dtype dt, double eps, const fct_params* prm_in, int32_t K, int32_t mode,
                     double* x, double* obj, int64_t* S, int32_t* status) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!b || !x || !status || !prm_in || K < 1 || d > 64 || (dt != FCT_F32 && dt != FCT_F64))
    return FCT_ERR_BAD_ARG;
  if (mode != FCT_SAMPLE_BERNOULLI && mode != FCT_SAMPLE_REPLACE) return FCT_ERR_BAD_ARG;
  fct_params prm = *prm_in;
  if (prm.s_out <= 0) {
    if (!(eps > 0.0)) return FCT_ERR_BAD_ARG;
    prm.s_out = (int64_t)std::ceil(20.0 * (d + 1) / eps);
  }
  if ((st = check_params(&prm, d + 1))) return st;
  const int iters = prm.irls_iters > 0 ? prm.irls_iters : 80;
  const int q = d + 1;
  int64_t cap;
  if (mode == FCT_SAMPLE_REPLACE) {
    cap = prm.s_out;
  } else {
    cap = 2 * prm.s_out + 8 * (int64_t)std::sqrt((double)prm.s_out) + 1024;
    if (cap > n) cap = n;
  }
  const size_t es = esize(dt);
  const int64_t n_pad = (n + prm.s - 1) / prm.s * prm.s;
  int perr = 0;
  const Pass1Plan plan = make_pass1_plan(c, n_pad, q, prm.s, prm.r1, es, prm.flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  // one sampling pass: R, lambda, sum lambda; then K draws, each with its
  // coreset, and the solver's arguments, outputs and work
  const int nwg = alike_solve_wgs(c, K, cap);
  auto layout = [&](auto& cv) {
    cv.template take<double>((size_t)q * q);
    cv.template take<float>((size_t)n);
    cv.template take<double>(1);
    cv.template take<int64_t>((size_t)K);
    cv.template take<char>(solve_args_bytes(K, nwg));
    cv.template take<double>((size_t)K * 72);
    for (int k = 0; k < K; ++k) {
      cv.template take<char>((size_t)cap * d * es);
      cv.template take<char>((size_t)cap * es);
      cv.template take<double>((size_t)cap);
      cv.template take<int64_t>((size_t)cap);
      cv.template take<double>(irls_batched_work_doubles(d, nwg));
      cv.template take<double>(72);
      cv.template take<int>(4);
    }
    if (mode == FCT_SAMPLE_REPLACE) carve_rep(cv, n);
  };
  Measure m;
  layout(m);
  const size_t fixed = m.off;
  Measure ma, mb, mc;
  carve_sketch(ma, plan, n_pad, q, prm.r1, es, true);
  carve_probs(mb, c, q, prm.r2, n, dt == FCT_F64 ? kPass2F64 : kPass2F32);
  carve_select(mc, n);
  const size_t rest = std::max(ma.off, std::max(mb.off, mc.off)) + 1024;
  if ((st = ensure_scratch(c, fixed + rest + 256))) return st;
  const size_t pin = std::max(solve_args_bytes(K, nwg), (size_t)K * 72 * sizeof(double));
  if ((st = batch_ensure_aux(c, pin))) return st;
  Carve cv(c->scratch);
  double* R = cv.take<double>((size_t)q * q);
  float* lam = cv.take<float>((size_t)n);
  double* sl = cv.take<double>(1);
  int64_t* S_dev = cv.take<int64_t>((size_t)K);
  IrlsArgs* args_dev = reinterpret_cast<IrlsArgs*>(cv.take<char>(solve_args_bytes(K, nwg)));
  double* out_dev = cv.take<double>((size_t)K * 72);
  std::vector<IrlsArgs> args((size_t)K);
  std::vector<int64_t*> idx((size_t)K);
  for (int k = 0; k < K; ++k) {
    IrlsArgs& a = args[k];
    a.At = cv.take<char>((size_t)cap * d * es);
    a.bt = cv.take<char>((size_t)cap * es);
    a.w = cv.take<double>((size_t)cap);
    idx[k] = cv.take<int64_t>((size_t)cap);
    double* work = cv.take<double>(irls_batched_work_doubles(d, nwg));
    double* outv = cv.take<double>(72);
    a.status = cv.take<int>(4);
    a.S_dev = S_dev + k;
    a.cap = cap;
    a.ldat = cap;
    a.d = d;
    a.iters = iters;
    a.row_target = solve_row_target(cap, nwg);
    a.part = work;
    a.bar = irls_batched_bar(work, d, nwg);
    a.x_out = outv;
    a.obj_out = outv + 64;
  }
  RepCdf rep{};
  if (mode == FCT_SAMPLE_REPLACE) rep = take_rep(cv, n);
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_sketch(c, sub, A, n, d, lda, dt, b, prm.s, prm.r1, prm.seed, prm.flags, nullptr,
                         R, nullptr, plan)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_probs(c, sub, A, b, n, d, lda, dt, R, prm.r2, prm.seed, lam, sl, prm.flags)))
      return st;
  }
  for (int k = 0; k < K; ++k) {
    double* w = const_cast<double*>(args[k].w);
    if (mode == FCT_SAMPLE_REPLACE) {
      HIP_TRY(launch_select_replace(lam, n, prm.s_out, prm.seed, (uint32_t)k, rep.bs, rep.pre,
                                    rep.cs, rep.co, rep.tot, k == 0, idx[k], w, S_dev + k,
                                    c->stream));
    } else {
      Carve sub(cv.base);
      sub.off = cv.off;
      if ((st = run_select(c, sub, lam, sl, n, (double)prm.s_out, prm.seed, cap, idx[k], w,
                           S_dev + k, (uint32_t)k)))
        return st;
    }
    HIP_TRY(launch_gather(A, b, lda, d, 1, n, idx[k], S_dev + k, cap, const_cast<void*>(args[k].At),
                          const_cast<void*>(args[k].bt), cap, dt == FCT_F64, c->stream));
  }
  if ((st = upload_solve_args(c, args, nwg, args_dev))) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));  // the pinned block is reused for the outputs
  prof_begin(c, 2);
  HIP_TRY(launch_solve_alike(args_dev, K, dt == FCT_F64, c->stream, nwg));
  prof_end(c, 2);
  hipLaunchKernelGGL(batch_collect_kernel, dim3(K), dim3(64), 0, c->stream, args_dev, K, out_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->bpinned, out_dev, (size_t)K * 72 * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);
  const double* h = reinterpret_cast<const double*>(c->bpinned);
  int first = FCT_OK;
  for (int k = 0; k < K; ++k) {
    const double* row = h + (size_t)k * 72;
    const int64_t Sk = (int64_t)row[65];
    int stk = (int)row[66];
    if (Sk > cap) stk = FCT_ERR_CAPACITY;
    status[k] = stk;
    for (int i = 0; i < d; ++i) x[(size_t)k * d + i] = row[i];
    if (obj) obj[k] = row[64];
    if (S) S[k] = Sk;
    if (stk != FCT_OK && first == FCT_OK) first = stk;
  }
  if (fl) return fl;
  return first;
}

int fct_l1_objectives(fct_ctx* c, const void* A, const void* B, int64_t n, int32_t d, int32_t k,
                      int64_t lda, int64_t ldb, fct_dtype dt, const double* W, double* out) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!W || !out || k < 1 || d > 64 || k > 64 || (dt != FCT_F32 && dt != FCT_F64)) return FCT_ERR_BAD_ARG;
  if (B && ldb < n) return FCT_ERR_BAD_ARG;
  const int nparts = 512;
  Measure m;
  m.take<double>((size_t)d * k);
  m.take<double>((size_t)nparts * k);
  m.take<double>((size_t)k);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  double* Wd = cv.take<double>((size_t)d * k);
  double* parts = cv.take<double>((size_t)nparts * k);
  double* res = cv.take<double>((size_t)k);
  // W (at most 64 x 64 doubles) through the resizable pinned block
  if ((st = batch_ensure_aux(c, (size_t)d * k * sizeof(double)))) return st;
  std::memcpy(c->bpinned, W, (size_t)d * k * sizeof(double));
  HIP_TRY(hipMemcpyAsync(Wd, c->bpinned, (size_t)d * k * sizeof(double), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(launch_l1_objectives(A, B, lda, ldb, n, d, k, Wd, dt == FCT_F64, parts, nparts, res,
                               c->stream));
  HIP_TRY(hipMemcpyAsync(c->bpinned, res, (size_t)k * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  const int fl = read_flags(c);
  std::memcpy(out, c->bpinned, (size_t)k * sizeof(double));
  return fl;
}

int l1_regress_mrhs(fct_ctx* c, const void* A, const void* B, int64_t n, int32_t d, int32_t k,
                    int64_t lda, int64_t ldb, fct_dtype dt, double eps, const fct_params* prm_in,
                    double* W, double* obj, int64_t* S_out, int32_t* status, double* R_out,
                    float* lambda_out) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!B || !W || !status || !prm_in || k < 1 || d > 64 || ldb < n ||
      (dt != FCT_F32 && dt != FCT_F64))
    return FCT_ERR_BAD_ARG;
  const int q = d + k;
  if (q > 88) return FCT_ERR_BAD_ARG;
  fct_params prm = *prm_in;
  if (prm.s_out <= 0) {
    if (!(eps > 0.0)) return FCT_ERR_BAD_ARG;
    prm.s_out = (int64_t)std::ceil(20.0 * q / eps);
  }
  if ((st = check_params(&prm, q))) return st;
  const int iters = prm.irls_iters > 0 ? prm.irls_iters : 80;
  int64_t cap = 2 * prm.s_out + 8 * (int64_t)std::sqrt((double)prm.s_out) + 1024;
  if (cap > n) cap = n;
  const size_t es = esize(dt);
  const int64_t n_pad = (n + prm.s - 1) / prm.s * prm.s;
  int perr = 0;
  const Pass1Plan plan = make_pass1_plan(c, n_pad, q, prm.s, prm.r1, es, prm.flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  const int nwg = alike_solve_wgs(c, k, cap);
  auto layout = [&](auto& cv) {
    cv.template take<double>((size_t)q * q);
    cv.template take<float>((size_t)n);
    cv.template take<double>(1);
    cv.template take<int64_t>(1);
    cv.template take<char>((size_t)cap * d * es);
    cv.template take<char>((size_t)cap * k * es);
    cv.template take<double>((size_t)cap);
    cv.template take<int64_t>((size_t)cap);
    cv.template take<char>(solve_args_bytes(k, nwg));
    cv.template take<double>((size_t)k * 72);
    for (int j = 0; j < k; ++j) {
      cv.template take<double>(irls_batched_work_doubles(d, nwg));
      cv.template take<double>(72);
      cv.template take<int>(4);
    }
  };
  Measure m;
  layout(m);
  Measure ma, mb, mc;
  carve_sketch(ma, plan, n_pad, q, prm.r1, es, true);
  carve_probs(mb, c, q, prm.r2, n, dt == FCT_F64 ? kPass2F64 : kPass2F32);
  carve_select(mc, n);
  if ((st = ensure_scratch(c, m.off + std::max(ma.off, std::max(mb.off, mc.off)) + 1280))) return st;
  const size_t pin = std::max(solve_args_bytes(k, nwg), (size_t)k * 72 * sizeof(double));
  if ((st = batch_ensure_aux(c, pin))) return st;
  Carve cv(c->scratch);
  double* R = cv.take<double>((size_t)q * q);
  float* lam = cv.take<float>((size_t)n);
  double* sl = cv.take<double>(1);
  int64_t* S_dev = cv.take<int64_t>(1);
  char* At = cv.take<char>((size_t)cap * d * es);
  char* Bt = cv.take<char>((size_t)cap * k * es);
  double* w = cv.take<double>((size_t)cap);
  int64_t* idx = cv.take<int64_t>((size_t)cap);
  IrlsArgs* args_dev = reinterpret_cast<IrlsArgs*>(cv.take<char>(solve_args_bytes(k, nwg)));
  double* out_dev = cv.take<double>((size_t)k * 72);
  std::vector<IrlsArgs> args((size_t)k);
  for (int j = 0; j < k; ++j) {
    IrlsArgs& a = args[j];
    double* work = cv.take<double>(irls_batched_work_doubles(d, nwg));
    double* outv = cv.take<double>(72);
    a.status = cv.take<int>(4);
    a.At = At;
    a.bt = Bt + (size_t)j * cap * es;
    a.w = w;
    a.S_dev = S_dev;
    a.cap = cap;
    a.ldat = cap;
    a.d = d;
    a.iters = iters;
    a.row_target = solve_row_target(cap, nwg);
    a.part = work;
    a.bar = irls_batched_bar(work, d, nwg);
    a.x_out = outv;
    a.obj_out = outv + 64;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_sketch(c, sub, A, n, d, lda, dt, B, prm.s, prm.r1, prm.seed, prm.flags, nullptr,
                         R, nullptr, plan, 0, k, ldb)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_probs(c, sub, A, B, n, d, lda, dt, R, prm.r2, prm.seed, lam, sl, prm.flags, k,
                        ldb)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_select(c, sub, lam, sl, n, (double)prm.s_out, prm.seed, cap, idx, w, S_dev)))
      return st;
  }
  HIP_TRY(launch_gather(A, B, lda, d, k, ldb, idx, S_dev, cap, At, Bt, cap, dt == FCT_F64,
                        c->stream));
  if (R_out)
    HIP_TRY(hipMemcpyAsync(R_out, R, (size_t)q * q * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  if (lambda_out)
    HIP_TRY(hipMemcpyAsync(lambda_out, lam, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice,
                           c->stream));
  if ((st = upload_solve_args(c, args, nwg, args_dev))) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_begin(c, 2);
  HIP_TRY(launch_solve_alike(args_dev, k, dt == FCT_F64, c->stream, nwg));
  prof_end(c, 2);
  hipLaunchKernelGGL(batch_collect_kernel, dim3(k), dim3(64), 0, c->stream, args_dev, k, out_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->bpinned, out_dev, (size_t)k * 72 * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  const int fl = read_flags(c);
  const double* h = reinterpret_cast<const double*>(c->bpinned);
  int first = FCT_OK;
  const int64_t S = (int64_t)h[65];
  if (S_out) *S_out = S;
  for (int j = 0; j < k; ++j) {
    const double* row = h + (size_t)j * 72;
    int stj = (int)row[66];
    if (S > cap) stj = FCT_ERR_CAPACITY;
    status[j] = stj;
    for (int i = 0; i < d; ++i) W[(size_t)j * d + i] = row[i];
    if (obj) obj[j] = row[64];
    if (stj != FCT_OK && first == FCT_OK) first = stj;
  }
  if (fl) return fl;
  return first;
}

int l1_subspace(fct_ctx* c, const void* A, int64_t n, int32_t d, int64_t lda, fct_dtype dt,
                double eps, const fct_params* prm_in, double* W, double* err, int32_t* j_star,
                int64_t* S_out, int32_t* status, double* R_out, float* lambda_out) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!W || !err || !j_star || !status || !prm_in || d < 2 || d > 64 ||
      (dt != FCT_F32 && dt != FCT_F64))
    return FCT_ERR_BAD_ARG;
  const int q = d;
  fct_params prm = *prm_in;
  if (prm.s_out <= 0) {
    if (!(eps > 0.0)) return FCT_ERR_BAD_ARG;
    prm.s_out = (int64_t)std::ceil(20.0 * q / eps);
  }
  if ((st = check_params(&prm, q))) return st;
  const int iters = prm.irls_iters > 0 ? prm.irls_iters : 80;
  int64_t cap = 2 * prm.s_out + 8 * (int64_t)std::sqrt((double)prm.s_out) + 1024;
  if (cap > n) cap = n;
  const size_t es = esize(dt);
  const int64_t n_pad = (n + prm.s - 1) / prm.s * prm.s;
  int perr = 0;
  const Pass1Plan plan = make_pass1_plan(c, n_pad, q, prm.s, prm.r1, es, prm.flags, &perr);
  if (perr) return FCT_ERR_BAD_ARG;
  const int dj = d - 1;
  const int nwg = alike_solve_wgs(c, d, cap);
  auto layout = [&](auto& cv) {
    cv.template take<double>((size_t)q * q);
    cv.template take<float>((size_t)n);
    cv.template take<double>(1);
    cv.template take<int64_t>(1);
    cv.template take<char>((size_t)cap * d * es);
    cv.template take<char>((size_t)cap * dj * d * es);
    cv.template take<char>((size_t)cap * d * es);
    cv.template take<double>((size_t)cap);
    cv.template take<int64_t>((size_t)cap);
    cv.template take<char>(solve_args_bytes(d, nwg));
    cv.template take<double>((size_t)d * 72);
    for (int j = 0; j < d; ++j) {
      cv.template take<double>(irls_batched_work_doubles(dj, nwg));
      cv.template take<double>(72);
      cv.template take<int>(4);
    }
  };
  Measure m;
  layout(m);
  Measure ma, mb, mc;
  carve_sketch(ma, plan, n_pad, q, prm.r1, es, true);
  carve_probs(mb, c, q, prm.r2, n, dt == FCT_F64 ? kPass2F64 : kPass2F32);
  carve_select(mc, n);
  if ((st = ensure_scratch(c, m.off + std::max(ma.off, std::max(mb.off, mc.off)) + 1280))) return st;
  const size_t pin = std::max(solve_args_bytes(d, nwg), (size_t)d * 72 * sizeof(double));
  if ((st = batch_ensure_aux(c, pin))) return st;
  Carve cv(c->scratch);
  double* R = cv.take<double>((size_t)q * q);
  float* lam = cv.take<float>((size_t)n);
  double* sl = cv.take<double>(1);
  int64_t* S_dev = cv.take<int64_t>(1);
  char* At = cv.take<char>((size_t)cap * d * es);
  char* Aj = cv.take<char>((size_t)cap * dj * d * es);
  char* bj = cv.take<char>((size_t)cap * d * es);
  double* w = cv.take<double>((size_t)cap);
  int64_t* idx = cv.take<int64_t>((size_t)cap);
  IrlsArgs* args_dev = reinterpret_cast<IrlsArgs*>(cv.take<char>(solve_args_bytes(d, nwg)));
  double* out_dev = cv.take<double>((size_t)d * 72);
  std::vector<IrlsArgs> args((size_t)d);
  for (int j = 0; j < d; ++j) {
    IrlsArgs& a = args[j];
    double* work = cv.take<double>(irls_batched_work_doubles(dj, nwg));
    double* outv = cv.take<double>(72);
    a.status = cv.take<int>(4);
    a.At = Aj + (size_t)j * cap * dj * es;
    a.bt = bj + (size_t)j * cap * es;
    a.w = w;
    a.S_dev = S_dev;
    a.cap = cap;
    a.ldat = cap;
    a.d = dj;
    a.iters = iters;
    a.row_target = solve_row_target(cap, nwg);
    a.part = work;
    a.bar = irls_batched_bar(work, dj, nwg);
    a.x_out = outv;
    a.obj_out = outv + 64;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_sketch(c, sub, A, n, d, lda, dt, nullptr, prm.s, prm.r1, prm.seed, prm.flags,
                         nullptr, R, nullptr, plan)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_probs(c, sub, A, nullptr, n, d, lda, dt, R, prm.r2, prm.seed, lam, sl,
                        prm.flags)))
      return st;
  }
  {
    Carve sub(cv.base);
    sub.off = cv.off;
    if ((st = run_select(c, sub, lam, sl, n, (double)prm.s_out, prm.seed, cap, idx, w, S_dev)))
      return st;
  }
  HIP_TRY(launch_gather(A, nullptr, lda, d, 0, n, idx, S_dev, cap, At, nullptr, cap,
                        dt == FCT_F64, c->stream));
  HIP_TRY(launch_drop_column(At, cap, d, S_dev, Aj, bj, dt == FCT_F64, c->stream));
  if (R_out)
    HIP_TRY(hipMemcpyAsync(R_out, R, (size_t)q * q * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  if (lambda_out)
    HIP_TRY(hipMemcpyAsync(lambda_out, lam, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice,
                           c->stream));
  if ((st = upload_solve_args(c, args, nwg, args_dev))) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  prof_begin(c, 2);
  HIP_TRY(launch_solve_alike(args_dev, d, dt == FCT_F64, c->stream, nwg));
  prof_end(c, 2);
  hipLaunchKernelGGL(batch_collect_kernel, dim3(d), dim3(64), 0, c->stream, args_dev, d, out_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->bpinned, out_dev, (size_t)d * 72 * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  int fl = read_flags(c);
  if (fl) return fl;
  const double* h = reinterpret_cast<const double*>(c->bpinned);
  int first = FCT_OK;
  const int64_t S = (int64_t)h[65];
  if (S_out) *S_out = S;
  // column j of W: the solution of regression j with -1 inserted at row j
  for (int j = 0; j < d; ++j) {
    const double* row = h + (size_t)j * 72;
    int stj = (int)row[66];
    if (S > cap) stj = FCT_ERR_CAPACITY;
    status[j] = stj;
    for (int i = 0, o = 0; i < d; ++i) W[(size_t)j * d + i] = i == j ? -1.0 : row[o++];
    if (stj != FCT_OK && first == FCT_OK) first = stj;
  }
  // the error of every candidate hyperplane over all rows: ||A w_j||_1
  if ((st = fct_l1_objectives(c, A, nullptr, n, d, d, lda, n, dt, W, err))) return st;
  int best = 0;
  for (int j = 1; j < d; ++j)
    if (err[j] < err[best]) best = j;
  *j_star = best;
  return first;
}

int fct_rng_words(fct_ctx* c, uint32_t stream, uint64_t seed, uint64_t idx0, int64_t count,
                  uint32_t* words) {
  if (!c || !words || count < 0 || stream > 6) return FCT_ERR_BAD_ARG;
  if (count == 0) return FCT_OK;
  HIP_TRY(launch_rng_words(stream, seed, idx0, count, words, c->stream));
  return FCT_OK;
}

int fct_pi1_streams(fct_ctx* c, uint64_t seed, int32_t r1, int32_t s, uint64_t j0, int64_t count,
                    int32_t* bh, float* ch, int32_t* bi, float* ci, int8_t* sg) {
  if (!c || r1 < 1 || count < 0 || !bh || !ch || !bi || !ci || !sg) return FCT_ERR_BAD_ARG;
  if (!is_pow2(s) || s < 2 || s > 4096) return FCT_ERR_BAD_ARG;
  if (count == 0) return FCT_OK;
  HIP_TRY(launch_pi1_streams(seed, (uint32_t)r1, ilog2(s), j0, count, bh, ch, bi, ci, sg,
                             c->stream));
  return FCT_OK;
}

int fct_fwht(fct_ctx* c, float* x, int64_t nblocks, int32_t s) {
  if (!c || !x || nblocks < 0 || !is_pow2(s) || s < 2 || s > 4096) return FCT_ERR_BAD_ARG;
  if (nblocks == 0) return FCT_OK;
  HIP_TRY(launch_fwht(x, nblocks, s, ilog2(s), c->stream));
  return FCT_OK;
}

int fct_to_bf16(fct_ctx* c, const float* x, int64_t count, uint16_t* y) {
  if (!c || !x || !y || count < 0) return FCT_ERR_BAD_ARG;
  if (count == 0) return FCT_OK;
  HIP_TRY(launch_to_bf16(x, count, y, c->stream));
  return FCT_OK;
}

int fct_lowp_residual(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
                      fct_dtype dt, const double* R, uint16_t* r_lowp, double* R_res) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!b || !R || !r_lowp || !R_res || d > 64 || (dt != FCT_F32 && dt != FCT_F64))
    return FCT_ERR_BAD_ARG;
  Measure m;
  m.take<double>(64);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  double* x0 = cv.take<double>(64);
  HIP_TRY(launch_lowp_residual(A, b, lda, n, d, dt == FCT_F64, R, x0, R_res, r_lowp, c->stream));
  return FCT_OK;
}

int fct_l1_objective(fct_ctx* c, const void* A, const void* b, int64_t n, int32_t d, int64_t lda,
                     fct_dtype dt, const double* x, double* out) {
  int st = check_common(c, A, n, d, lda);
  if (st) return st;
  if (!b || !x || !out || d > 64 || (dt != FCT_F32 && dt != FCT_F64)) return FCT_ERR_BAD_ARG;
  const int nparts = 1024;
  Measure m;
  m.take<double>(64);
  m.take<double>(nparts);
  m.take<double>(1);
  if ((st = ensure_scratch(c, m.off))) return st;
  Carve cv(c->scratch);
  double* xd = cv.take<double>(64);
  double* parts = cv.take<double>(nparts);
  double* res = cv.take<double>(1);
  std::memcpy((char*)c->pinned + 2048, x, d * sizeof(double));
  HIP_TRY(hipMemcpyAsync(xd, (char*)c->pinned + 2048, d * sizeof(double), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(launch_l1_objective(A, b, lda, n, d, xd, dt == FCT_F64, parts, nparts, res, c->stream));
  HIP_TRY(hipMemcpyAsync(c->pinned, res, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(out, c->pinned, sizeof(double));
  return FCT_OK;
}

}  // extern "C"
