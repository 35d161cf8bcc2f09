// Steps 6-7 of the regression figure: p_i = min{1, s lambda_i / sum lambda},
// D_ii = 1/p_i with probability p_i, and the rows with D_ii != 0 gathered
// into the coreset (O(n) to draw D, O(q S) to form D A and D b).
//
// Row i is kept iff its stream-3 word w_i satisfies w_i < floor(p_i 2^32),
// with p_i formed in FP64 (the event "uniform < p_i" on the 2^-32 grid).
// Kept rows are listed in ascending order by one pass over lambda: a
// workgroup takes the next 16384-row tile from a ticket counter, decides its
// rows, publishes its count, and finds the count of all earlier tiles by
// looking back over their published counts and prefixes (a decoupled
// look-back scan); then it writes its rows at that offset after an in-tile
// prefix sum.  Tiles are handed out in ticket order, so every tile a
// workgroup waits for belongs to a workgroup that is already running.
#include "../../include/fctl1.h"
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

static constexpr int kSelThreads = 256;
static constexpr int kSelRowsPerThread = 64;
static constexpr int kSelRows = kSelThreads * kSelRowsPerThread;

int select_grid(int64_t n) { return (int)((n + kSelRows - 1) / kSelRows); }

__device__ __forceinline__ uint64_t threshold(float lam, double s_out, double total, double* p) {
  double pv = total > 0.0 ? s_out * (double)lam / total : 1.0;
  pv = pv < 1.0 ? pv : 1.0;
  *p = pv;
  const double t = floor(pv * 4294967296.0);
  return (uint64_t)(t < 4294967296.0 ? t : 4294967296.0);
}

// Keep mask of this thread's 64 consecutive rows (bit k = row base + k);
// base is a multiple of 64, so a whole group is sixteen 16-byte loads.  The
// decision w < floor(p 2^32) holds iff the unfloored p 2^32 >= w + 1.  That
// value is first estimated as lambda * (s_out 2^32 / sum lambda), within a few
// units of 2^-53 of it; the estimate settles the decision unless it lies
// within a relative 1e-12 of w + 1, and only those rare rows (and every row
// when p is written out) evaluate p itself as the oracle does.
__device__ __forceinline__ uint64_t keep_mask(const SelectArgs& a, int64_t base, double total,
                                              bool write_p) {
  float lam[kSelRowsPerThread];
  if (base + kSelRowsPerThread <= a.n) {
    const float4* l4 = reinterpret_cast<const float4*>(a.lambda + base);
#pragma unroll
    for (int k = 0; k < kSelRowsPerThread / 4; ++k) {
      const float4 x = l4[k];
      lam[4 * k + 0] = x.x;
      lam[4 * k + 1] = x.y;
      lam[4 * k + 2] = x.z;
      lam[4 * k + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSelRowsPerThread; ++k) lam[k] = base + k < a.n ? a.lambda[base + k] : 0.0f;
  }
  const bool quick = !write_p && total > 0.0;
  const double scale = quick ? a.s_out * 4294967296.0 / total : 0.0;
  uint64_t mask = 0;
#pragma unroll
  for (int qd = 0; qd < kSelRowsPerThread / 4; ++qd) {
    const int64_t r0 = base + 4 * qd;
    if (r0 >= a.n) break;
    const uint4 w = stream_words(a.seed, kStreamSample, (uint64_t)r0 >> 2, a.instance);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = r0 + k;
      if (i < a.n) {
        const double need = (double)ws[k] + 1.0;
        const double est = (double)lam[4 * qd + k] * scale;
        bool keep;
        if (quick && (est > need * (1.0 + 1e-12) || est < need * (1.0 - 1e-12))) {
          keep = est > need;
        } else {
          double p;
          const uint64_t t = threshold(lam[4 * qd + k], a.s_out, total, &p);
          if (write_p && a.p_out) a.p_out[i] = (float)p;
          keep = (uint64_t)ws[k] < t;
        }
        if (keep) mask |= 1ull << (4 * qd + k);
      }
    }
  }
  return mask;
}

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  // sh: kSelThreads / 64 + 1 ints
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kSelThreads / 64; ++w) {
      const int t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[kSelThreads / 64] = run;
  }
  __syncthreads();
  *total = sh[kSelThreads / 64];
  return sh[wave] + x - v;
}

// Look-back status of a tile: the count of kept rows in the low 62 bits,
// flag kAgg once the tile's own count is published, kPre once the count of
// all tiles up to and including it is.
constexpr uint64_t kAgg = 1ull << 62, kPre = 2ull << 62, kCountMask = (1ull << 62) - 1;
// a wait longer than about a second means a tile will never be published:
// the pass stops and reports FCT_ERR_HIP instead of waiting for ever
constexpr uint32_t kLookbackSpins = 1u << 22;

// The status word carries everything a reader needs (flag and count in one
// 64-bit atomic), so the accesses are relaxed: agent-scope atomics that go
// to the coherent cache level, without the whole-cache write-back and
// invalidation that release and acquire ordering would add on every access.
__device__ __forceinline__ uint64_t load_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// status [nb] and the ticket counter status[nb] start at zero
__global__ void select_init_kernel(uint64_t* __restrict__ status, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= nb) status[i] = 0ull;
}

__global__ void __launch_bounds__(kSelThreads) select_kernel(SelectArgs a, int nb) {
  __shared__ int sh[kSelThreads / 64 + 1];
  __shared__ int s_tile;
  __shared__ int64_t s_before;
  uint64_t* status = a.lookback;
  if (threadIdx.x == 0)
    s_tile = (int)__hip_atomic_fetch_add(&status[nb], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int tile = s_tile;
  const double total = *a.sum_lambda;
  const int64_t base = (int64_t)tile * kSelRows + (int64_t)threadIdx.x * kSelRowsPerThread;
  uint64_t m = keep_mask(a, base, total, a.p_out != nullptr);
  int tot;
  const int pre = block_exclusive_scan(__popcll(m), sh, &tot);

  if (threadIdx.x < 64) {
    // wave 0: publish, then add the counts of the tiles before this one,
    // 64 at a time (lane l looks at tile j - l), up to the nearest prefix
    const int lane = threadIdx.x;
    int64_t before = 0;
    if (tile == 0) {
      if (lane == 0) store_status(&status[0], kPre | (uint64_t)tot);
    } else {
      if (lane == 0) store_status(&status[tile], kAgg | (uint64_t)tot);
      int64_t j = tile - 1;
      uint32_t spins = 0;
      bool failed = false;
      for (;;) {
        const int64_t t = j - lane;
        uint64_t v = t >= 0 ? load_status(&status[t]) : kPre;  // nothing before tile 0
        while (__ballot((v >> 62) == 0)) {
          if (++spins > kLookbackSpins) {
            failed = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          if ((v >> 62) == 0) v = load_status(&status[t]);
        }
        if (failed) break;
        const unsigned long long pm = __ballot((v >> 62) == 2);
        const int k = pm ? __ffsll((long long)pm) - 1 : 63;  // nearest tile with a prefix
        int64_t mine = lane <= k ? (int64_t)(v & kCountMask) : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mine += __shfl_xor(mine, o, 64);
        before += mine;
        if (pm) break;
        j -= 64;
      }
      if (failed) {
        if (lane == 0) atomicCAS(a.fail, 0, (int)FCT_ERR_HIP);
        before = 0;
      }
      if (lane == 0) store_status(&status[tile], kPre | (uint64_t)(before + tot));
    }
    if (lane == 0) s_before = before;
  }
  __syncthreads();
  const int64_t first = s_before;
  if (tile == nb - 1 && threadIdx.x == 0) *a.S = first + tot;
  int64_t pos = first + pre;
  while (m) {
    const int k = __ffsll((long long)m) - 1;
    m &= m - 1;
    const int64_t i = base + k;
    if (pos < a.cap) {
      double p;
      threshold(a.lambda[i], a.s_out, total, &p);
      a.idx[pos] = i;
      a.w[pos] = 1.0 / p;
    }
    ++pos;
  }
}

hipError_t launch_select(const SelectArgs& a, hipStream_t st) {
  const int nb = select_grid(a.n);
  hipLaunchKernelGGL(select_init_kernel, dim3((unsigned)((nb + 256) / 256)), dim3(256), 0, st,
                     a.lookback, nb);
  hipLaunchKernelGGL(select_kernel, dim3(nb), dim3(kSelThreads), 0, st, a, nb);
  return hipGetLastError();
}

// ---- sampling with replacement ---------------------------------------------
//
// Exactly s samples, independent, with probabilities lambda_i / sum lambda
// (the caption of the regression figure), by inversion of the running sums
// C of lambda: sample j takes the row i with C_(i-1) <= u_j C_n < C_i, u_j =
// (w_j + 1/2) / 2^32 from its stream-4 word.  C is held at the granularity of
// 256-row blocks (FP64 sums of 256 rows, their exclusive prefix in fixed-size
// chunks); a sample finds its block by binary search and its row by running
// the block's sum in row order.

static constexpr int kRepBlock = 256;   // rows per block sum
static constexpr int kRepChunk = 1024;  // block sums per scan chunk

int64_t rep_blocks(int64_t n) { return (n + kRepBlock - 1) / kRepBlock; }
int64_t rep_chunks(int64_t n) { return (rep_blocks(n) + kRepChunk - 1) / kRepChunk; }

// bs[b]: a wave per block, each lane its 4 consecutive rows in order, the
// lanes' sums by a fixed tree
__global__ void __launch_bounds__(256) rep_block_sums_kernel(const float* __restrict__ lam, int64_t n,
                                                             int64_t nb, double* __restrict__ bs) {
  const int lane = threadIdx.x & 63;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); blk < nb;
       blk += (int64_t)gridDim.x * 4) {
    const int64_t r = blk * kRepBlock + 4 * lane;
    double v = 0.0;
    if (r + 3 < n) {
      const float4 x = *reinterpret_cast<const float4*>(lam + r);
      v = (((double)x.x + (double)x.y) + (double)x.z) + (double)x.w;
    } else {
      for (int k = 0; k < 4; ++k)
        if (r + k < n) v += (double)lam[r + k];
    }
    v = wave_sum_dpp(v);
    if (lane == 0) bs[blk] = v;
  }
}

// cs[c]: the sum of bs over chunk c (each thread 4 in order, then a fixed tree)
__global__ void __launch_bounds__(256) rep_chunk_sums_kernel(const double* __restrict__ bs, int64_t nb,
                                                             double* __restrict__ cs) {
  __shared__ double red[4];
  const int64_t b0 = (int64_t)blockIdx.x * kRepChunk + 4 * threadIdx.x;
  double v = 0.0;
  for (int k = 0; k < 4; ++k)
    if (b0 + k < nb) v += bs[b0 + k];
  v = wave_sum_dpp(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) cs[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// one workgroup: co = exclusive prefix of cs (runs per thread in order, then
// the run totals in order); tot = the sum of everything
__global__ void __launch_bounds__(1024) rep_chunk_scan_kernel(const double* __restrict__ cs, int nc,
                                                              double* __restrict__ co,
                                                              double* __restrict__ tot) {
  __shared__ double run[1024];
  const int T = blockDim.x;
  const int per = (nc + T - 1) / T;
  const int lo = threadIdx.x * per, hi = min(nc, lo + per);
  double s = 0.0;
  for (int i = lo; i < hi; ++i) s += cs[i];
  run[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int t = 0; t < T; ++t) {
      const double v = run[t];
      run[t] = acc;
      acc += v;
    }
    *tot = acc;
  }
  __syncthreads();
  double o = run[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    co[i] = o;
    o += cs[i];
  }
}

// pre[b] = co[chunk] + the exclusive prefix of bs within the chunk (each
// thread 4 in order, the thread totals scanned in thread order)
__global__ void __launch_bounds__(256) rep_block_prefix_kernel(const double* __restrict__ bs, int64_t nb,
                                                               const double* __restrict__ co,
                                                               double* __restrict__ pre) {
  __shared__ double ts[256];
  const int64_t b0 = (int64_t)blockIdx.x * kRepChunk + 4 * threadIdx.x;
  double v[4], s = 0.0;
  for (int k = 0; k < 4; ++k) {
    v[k] = b0 + k < nb ? bs[b0 + k] : 0.0;
    s += v[k];
  }
  ts[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = co[blockIdx.x];
    for (int t = 0; t < 256; ++t) {
      const double x = ts[t];
      ts[t] = acc;
      acc += x;
    }
  }
  __syncthreads();
  double o = ts[threadIdx.x];
  for (int k = 0; k < 4; ++k)
    if (b0 + k < nb) {
      pre[b0 + k] = o;
      o += v[k];
    }
}

// one thread per sample: its block by binary search over pre (the last block
// whose prefix is <= the target: empty blocks are skipped), its row by the
// block's running sum; a target past the block's last running sum (the two
// sums rounded in another order) takes the block's last row with lambda > 0
__global__ void __launch_bounds__(256) rep_sample_kernel(const float* __restrict__ lam, int64_t n,
                                                         const double* __restrict__ pre, int64_t nb,
                                                         const double* __restrict__ tot, int64_t s,
                                                         uint64_t seed, uint32_t instance,
                                                         int64_t* __restrict__ idx,
                                                         double* __restrict__ w,
                                                         int64_t* __restrict__ S) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *S = s;
  if (j >= s) return;
  const uint4 wv = stream_words(seed, kStreamReplace, (uint64_t)j >> 2, instance);
  const uint32_t sel = (uint32_t)j & 3u;
  const uint32_t word = sel == 0 ? wv.x : sel == 1 ? wv.y : sel == 2 ? wv.z : wv.w;
  const double total = *tot;
  const double t = ((double)word + 0.5) * 0x1p-32 * total;
  int64_t lo = 0, hi = nb - 1;  // pre[0] = 0 <= t
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int64_t r0 = lo * kRepBlock, r1 = min(n, r0 + kRepBlock);
  double c = pre[lo];
  int64_t row = -1, last = r0;
  for (int64_t r = r0; r < r1; ++r) {
    const float v = lam[r];
    if (v > 0.0f) last = r;
    c += (double)v;
    if (t < c) {
      row = r;
      break;
    }
  }
  if (row < 0) row = last;
  idx[j] = row;
  w[j] = total / ((double)s * (double)lam[row]);
}

hipError_t launch_select_replace(const float* lambda, int64_t n, int64_t s, uint64_t seed,
                                 uint32_t instance, double* bs, double* pre, double* cs,
                                 double* co, double* tot, bool build_cdf, int64_t* idx, double* w,
                                 int64_t* S, hipStream_t st) {
  const int64_t nb = rep_blocks(n), nc = rep_chunks(n);
  if (build_cdf) {
    int64_t g = (nb + 3) / 4;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(rep_block_sums_kernel, dim3((unsigned)g), dim3(256), 0, st, lambda, n, nb, bs);
    hipLaunchKernelGGL(rep_chunk_sums_kernel, dim3((unsigned)nc), dim3(256), 0, st, bs, nb, cs);
    hipLaunchKernelGGL(rep_chunk_scan_kernel, dim3(1), dim3(1024), 0, st, cs, (int)nc, co, tot);
    hipLaunchKernelGGL(rep_block_prefix_kernel, dim3((unsigned)nc), dim3(256), 0, st, bs, nb, co, pre);
  }
  hipLaunchKernelGGL(rep_sample_kernel, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, lambda,
                     n, pre, nb, tot, s, seed, instance, idx, w, S);
  return hipGetLastError();
}

// probabilities only (l1_sample_probs with p requested)
__global__ void __launch_bounds__(256) probs_kernel(SelectArgs a) {
  const double total = *a.sum_lambda;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double p;
  threshold(a.lambda[i], a.s_out, total, &p);
  a.p_out[i] = (float)p;
}

hipError_t launch_probs_only(const SelectArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(probs_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
__global__ void gather_kernel(const T* __restrict__ A, const T* __restrict__ b, int64_t lda,
                              int32_t d, int32_t kb, int64_t ldb, const int64_t* __restrict__ idx,
                              const int64_t* __restrict__ S, int64_t cap, T* __restrict__ At,
                              T* __restrict__ bt, int64_t ldat) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cnt = min(*S, cap);
  if (k >= cnt) return;
  const int64_t i = idx[k];
  for (int c = 0; c < d; ++c) At[k + (int64_t)c * ldat] = A[i + (int64_t)c * lda];
  for (int c = 0; c < kb; ++c) bt[k + (int64_t)c * ldat] = b[i + (int64_t)c * ldb];
}

hipError_t launch_gather(const void* A, const void* b, int64_t lda, int32_t d, int32_t kb,
                         int64_t ldb, const int64_t* idx, const int64_t* S, int64_t cap, void* At,
                         void* bt, int64_t ldat, bool f64, hipStream_t st) {
  const unsigned grid = (unsigned)((cap + 255) / 256);
  if (!b) kb = 0;
  if (f64)
    hipLaunchKernelGGL(gather_kernel<double>, dim3(grid), dim3(256), 0, st, (const double*)A,
                       (const double*)b, lda, d, kb, ldb, idx, S, cap, (double*)At, (double*)bt,
                       ldat);
  else
    hipLaunchKernelGGL(gather_kernel<float>, dim3(grid), dim3(256), 0, st, (const float*)A,
                       (const float*)b, lda, d, kb, ldb, idx, S, cap, (float*)At, (float*)bt,
                       ldat);
  return hipGetLastError();
}

}  // namespace fctl1
