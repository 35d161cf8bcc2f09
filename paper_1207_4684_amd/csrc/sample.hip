// Steps 6-7 of the regression figure: p_i = min{1, s lambda_i / sum lambda},
// D_ii = 1/p_i with probability p_i, and the rows with D_ii != 0 gathered
// into the coreset (O(n) to draw D, O(q S) to form D A and D b).
//
// Row i is kept iff its stream-3 word w_i satisfies w_i < floor(p_i 2^32),
// with p_i formed in FP64 (the event "uniform < p_i" on the 2^-32 grid).
// Kept rows are listed in ascending order: a first kernel counts the kept
// rows of each 4096-row tile, one workgroup scans the counts, and a second
// pass writes each tile's rows at its offset after an in-tile prefix sum.
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

static constexpr int kSelThreads = 256;
static constexpr int kSelRowsPerThread = 16;
static constexpr int kSelRows = kSelThreads * kSelRowsPerThread;

int select_grid(int64_t n) { return (int)((n + kSelRows - 1) / kSelRows); }

__device__ __forceinline__ uint64_t threshold(float lam, double s_out, double total, double* p) {
  double pv = total > 0.0 ? s_out * (double)lam / total : 1.0;
  pv = pv < 1.0 ? pv : 1.0;
  *p = pv;
  const double t = floor(pv * 4294967296.0);
  return (uint64_t)(t < 4294967296.0 ? t : 4294967296.0);
}

// keep mask of this thread's 16 consecutive rows (bit k = row base + k)
__device__ __forceinline__ uint32_t keep_mask(const SelectArgs& a, int64_t base, double total,
                                              bool write_p) {
  uint32_t mask = 0;
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
        double p;
        const uint64_t t = threshold(a.lambda[i], a.s_out, total, &p);
        if (write_p && a.p_out) a.p_out[i] = (float)p;
        if ((uint64_t)ws[k] < t) mask |= 1u << (4 * qd + k);
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

__global__ void __launch_bounds__(kSelThreads) select_count_kernel(SelectArgs a) {
  __shared__ int sh[kSelThreads / 64 + 1];
  const double total = *a.sum_lambda;
  const int64_t base = (int64_t)blockIdx.x * kSelRows + (int64_t)threadIdx.x * kSelRowsPerThread;
  const uint32_t m = keep_mask(a, base, total, true);
  int tot;
  block_exclusive_scan(__popc(m), sh, &tot);
  if (threadIdx.x == 0) a.counts[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) scan_counts_kernel(const int32_t* __restrict__ counts,
                                                           int nb, int64_t* __restrict__ offsets,
                                                           int64_t* __restrict__ S) {
  // one workgroup: each thread sums a contiguous run, then a scan of run totals
  __shared__ int64_t run[1024];
  const int T = blockDim.x;
  const int per = (nb + T - 1) / T;
  const int lo = threadIdx.x * per, hi = min(nb, lo + per);
  int64_t s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  run[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int t = 0; t < T; ++t) {
      const int64_t v = run[t];
      run[t] = acc;
      acc += v;
    }
    offsets[nb] = acc;
    *S = acc;
  }
  __syncthreads();
  int64_t o = run[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    offsets[i] = o;
    o += counts[i];
  }
}

__global__ void __launch_bounds__(kSelThreads) select_write_kernel(SelectArgs a) {
  __shared__ int sh[kSelThreads / 64 + 1];
  const double total = *a.sum_lambda;
  const int64_t base = (int64_t)blockIdx.x * kSelRows + (int64_t)threadIdx.x * kSelRowsPerThread;
  uint32_t m = keep_mask(a, base, total, false);
  int tot;
  const int pre = block_exclusive_scan(__popc(m), sh, &tot);
  int64_t pos = a.offsets[blockIdx.x] + pre;
  while (m) {
    const int k = __ffs(m) - 1;
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
  hipLaunchKernelGGL(select_count_kernel, dim3(nb), dim3(kSelThreads), 0, st, a);
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(1024), 0, st, a.counts, nb, a.offsets, a.S);
  hipLaunchKernelGGL(select_write_kernel, dim3(nb), dim3(kSelThreads), 0, st, a);
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
                              int32_t d, const int64_t* __restrict__ idx,
                              const int64_t* __restrict__ S, int64_t cap, T* __restrict__ At,
                              T* __restrict__ bt, int64_t ldat) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cnt = min(*S, cap);
  if (k >= cnt) return;
  const int64_t i = idx[k];
  for (int c = 0; c < d; ++c) At[k + (int64_t)c * ldat] = A[i + (int64_t)c * lda];
  bt[k] = b[i];
}

hipError_t launch_gather(const void* A, const void* b, int64_t lda, int32_t d, const int64_t* idx,
                         const int64_t* S, int64_t cap, void* At, void* bt, int64_t ldat, bool f64,
                         hipStream_t st) {
  const unsigned grid = (unsigned)((cap + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(gather_kernel<double>, dim3(grid), dim3(256), 0, st, (const double*)A,
                       (const double*)b, lda, d, idx, S, cap, (double*)At, (double*)bt, ldat);
  else
    hipLaunchKernelGGL(gather_kernel<float>, dim3(grid), dim3(256), 0, st, (const float*)A,
                       (const float*)b, lda, d, idx, S, cap, (float*)At, (float*)bt, ldat);
  return hipGetLastError();
}

}  // namespace fctl1
