// Pass 1: Y = Pi1 X with the FCT1 transform Pi1 = 4 B C H~ (section "FCT1
// Construction"; running time O(n log s): n/s Hadamard transforms of size s,
// a diagonal Cauchy scaling and a hash scatter with 2n non-zeros).
//
// Work decomposition.  A workgroup owns a range of whole s-row blocks and a
// slice of c columns of X = [A, -b].  It keeps a private r1 x c accumulator in
// LDS (layout [bucket][column]) and walks its range in chunks of
// max(s, blockDim) rows:
//   A. each thread takes rows t, t + NT, ... of the chunk; one Philox call
//      per row gives both stacked positions' (bucket, Cauchy) pairs, kept in
//      registers for the whole chunk; the sign D(j) comes from words staged in
//      LDS; u = D x is stored to an LDS tile and its I-half contribution
//      4 C_I u is added into bucket h_I;
//   B. the tile is transformed in place: radix-16 butterfly passes in
//      registers over 4 index bits at a time (Sylvester order, H_s =
//      H_2 (x) ... (x) H_2 over the bits of the row index inside the block);
//   C. each thread reads back its rows and adds 4 C_H (H_s u)_t / sqrt(s)
//      into bucket h_H.
// The accumulator is written once per workgroup to a partial buffer; a
// second kernel sums the partials of each output element in a fixed order in
// FP64.  Rows past n are zero (padding to s ceil(n/s)); chunks past the last
// block are skipped.
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

__device__ __forceinline__ int tpad(int t) { return t + (t >> 4); }

template <typename T> __device__ __forceinline__ T cauchy_t(uint32_t w);
template <> __device__ __forceinline__ float cauchy_t<float>(uint32_t w) { return cauchy_from_word(w); }
template <> __device__ __forceinline__ double cauchy_t<double>(uint32_t w) {
  return cauchy_from_word_f64(w);
}

template <typename T, int R>
__device__ __forceinline__ void fwht_regs(T (&v)[R]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if ((i & h) == 0) {
        const T a = v[i], bb = v[i + h];
        v[i] = a + bb;
        v[i + h] = a - bb;
      }
    }
  }
}

// One radix-R pass over index bits [log2 st, log2 st + log2 R) of every
// column's chunk in the tile (column stride TP, padded row index).
template <typename T, int R>
__device__ __forceinline__ void fwht_pass(T* tile, int TP, int cs, int chunk, int st) {
  const int groups = chunk / R;
  const int gshift = __builtin_ctz(groups);
  const int sshift = __builtin_ctz(st);
  for (int task = threadIdx.x; task < cs * groups; task += blockDim.x) {
    const int col = task >> gshift;
    const int g = task & (groups - 1);
    const int base = ((g >> sshift) << (sshift + __builtin_ctz(R))) + (g & (st - 1));
    T* p = tile + col * TP;
    T v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = p[tpad(base + i * st)];
    fwht_regs<T, R>(v);
#pragma unroll
    for (int i = 0; i < R; ++i) p[tpad(base + i * st)] = v[i];
  }
}

template <typename T>
__device__ void fwht_tile(T* tile, int TP, int cs, int chunk, int log2s) {
  int lo = 0;
  while (lo < log2s) {
    const int rb = min(4, log2s - lo);
    const int st = 1 << lo;
    switch (rb) {
      case 4: fwht_pass<T, 16>(tile, TP, cs, chunk, st); break;
      case 3: fwht_pass<T, 8>(tile, TP, cs, chunk, st); break;
      case 2: fwht_pass<T, 4>(tile, TP, cs, chunk, st); break;
      default: fwht_pass<T, 2>(tile, TP, cs, chunk, st); break;
    }
    lo += rb;
    __syncthreads();
  }
}

template <typename T, int RPT>
__global__ void __launch_bounds__(1024) pass1_kernel(Pass1Args a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int NT = blockDim.x;
  const int chunk = NT * RPT;
  const int TP = chunk + (chunk >> 4);
  const int rr = blockIdx.x;
  const int c0 = blockIdx.y * a.c;
  const int cs = min(a.c, a.q - c0);
  T* acc = reinterpret_cast<T*>(smem_raw);
  T* tile = acc + (size_t)a.r1 * a.c;
  uint32_t* sgnw = reinterpret_cast<uint32_t*>(tile + (size_t)a.c * TP);

  for (int i = threadIdx.x; i < a.r1 * cs; i += NT) acc[i] = T(0);

  const int64_t row0 = (int64_t)rr * a.rows_per_range;
  const int64_t row1 = min(a.n_pad, row0 + a.rows_per_range);
  const T scale_h = T(4) / sqrt(T(a.s));
  const T scale_i = T(4);

  for (int64_t cr = row0; cr < row1; cr += chunk) {
    __syncthreads();  // previous chunk's tile reads and sign words are done
    if (a.sign_flip) {
      for (int k = threadIdx.x; k < chunk / 128; k += NT) {
        const uint4 w = stream_words(a.seed, kStreamSign, (uint64_t)((a.row0g + cr) >> 7) + k,
                                     a.instance);
        sgnw[4 * k + 0] = w.x;
        sgnw[4 * k + 1] = w.y;
        sgnw[4 * k + 2] = w.z;
        sgnw[4 * k + 3] = w.w;
      }
    }
    __syncthreads();

    uint32_t hH[RPT], hI[RPT];
    T cH[RPT], cI[RPT];
    bool valid[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int t = threadIdx.x + r * NT;
      const int64_t j = cr + t;
      valid[r] = j < row1;
      const uint64_t kH = h_position((uint64_t)(a.row0g + j), a.log2s);
      uint32_t bH, wH, bI, wI;
      position_words(a.seed, a.instance, kH, a.r1, &bH, &wH);
      position_words(a.seed, a.instance, kH + a.s, a.r1, &bI, &wI);
      hH[r] = bH * cs;
      cH[r] = cauchy_t<T>(wH) * scale_h;
      hI[r] = bI * cs;
      cI[r] = cauchy_t<T>(wI) * scale_i;
      float sg = 1.0f;
      if (a.sign_flip) {
        const uint32_t word = sgnw[t >> 5];
        sg = ((word >> (t & 31)) & 1u) ? -1.0f : 1.0f;
      }
      const bool inrange = j < a.n;
      for (int col = 0; col < cs; ++col) {
        const int gc = c0 + col;
        T x = T(0);
        if (inrange) {
          if (gc < a.d) x = reinterpret_cast<const T*>(a.A)[j + (int64_t)gc * a.lda];
          else x = -reinterpret_cast<const T*>(a.b)[j + (int64_t)(gc - a.d) * a.ldb];
        }
        const T u = T(sg) * x;
        tile[col * TP + tpad(t)] = u;
        if (valid[r]) atomicAdd(&acc[hI[r] + col], cI[r] * u);
      }
    }
    __syncthreads();
    fwht_tile<T>(tile, TP, cs, chunk, a.log2s);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int t = threadIdx.x + r * NT;
      if (!valid[r]) continue;
      for (int col = 0; col < cs; ++col) {
        const T v = tile[col * TP + tpad(t)];
        atomicAdd(&acc[hH[r] + col], cH[r] * v);
      }
    }
  }
  __syncthreads();
  T* part = reinterpret_cast<T*>(a.partials);
  for (int col = 0; col < cs; ++col) {
    T* dst = part + ((size_t)rr * a.q + c0 + col) * a.r1;
    for (int i = threadIdx.x; i < a.r1; i += NT) dst[i] = acc[i * cs + col];
  }
}

// Y (r1 x q column-major) = sum over ranges of the partials, FP64, in a
// fixed order: a workgroup takes 64 consecutive entries, its wave g adds the
// ranges g, g + 8, g + 16, ... in turn, and the eight wave sums are added in
// wave order.
constexpr int kRedGroups = 8;

template <typename T, typename TY>
__global__ void __launch_bounds__(64 * kRedGroups)
reduce_partials_kernel(const T* __restrict__ part, int nranges, int r1, int q,
                       TY* __restrict__ Y, double* __restrict__ Yd, int* __restrict__ flag) {
  __shared__ double ws[kRedGroups][64];
  const int i = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + i;
  const int64_t tot = (int64_t)r1 * q;
  double s = 0.0;
  if (idx < tot) {
    // eight of the wave's ranges are loaded before they are added (in the
    // same order), so that the loads are in flight together
    constexpr int U = 8;
    int rr = g;
    for (; rr + (U - 1) * kRedGroups < nranges; rr += U * kRedGroups) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = part[(size_t)(rr + u * kRedGroups) * tot + idx];
#pragma unroll
      for (int u = 0; u < U; ++u) s += (double)x[u];
    }
    for (; rr < nranges; rr += kRedGroups) s += (double)part[(size_t)rr * tot + idx];
  }
  ws[g][i] = s;
  __syncthreads();
  if (g != 0 || idx >= tot) return;
  s = ws[0][i];
#pragma unroll
  for (int k = 1; k < kRedGroups; ++k) s += ws[k][i];
  if (Yd) Yd[idx] = s;
  if (Y) Y[idx] = (TY)s;
  if (!isfinite(s)) *flag = 1;
}

template <typename T, int RPT>
static hipError_t launch_pass1_t(const Pass1Args& a, const Pass1Plan& p, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)pass1_kernel<T, RPT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((pass1_kernel<T, RPT>), dim3(p.nranges, p.nslices), dim3(p.threads), p.lds,
                     st, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pass1_rpt(const Pass1Args& a, const Pass1Plan& p, hipStream_t st) {
  switch (p.rpt) {
    case 1: return launch_pass1_t<T, 1>(a, p, st);
    case 2: return launch_pass1_t<T, 2>(a, p, st);
    case 4: return launch_pass1_t<T, 4>(a, p, st);
    case 8: return launch_pass1_t<T, 8>(a, p, st);
    case 16: return launch_pass1_t<T, 16>(a, p, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass1(const Pass1Args& a, const Pass1Plan& p, bool f64, hipStream_t st) {
  if (f64) return launch_pass1_rpt<double>(a, p, st);
  return launch_pass1_rpt<float>(a, p, st);
}

hipError_t launch_reduce_partials(const void* part, int nranges, int r1, int q, void* Y,
                                  double* Yd, int* flag, bool f64, hipStream_t st, int y_f64) {
  const int64_t tot = (int64_t)r1 * q;
  const int threads = 64 * kRedGroups;
  const int blocks = (int)((tot + 63) / 64);
  const bool yd = y_f64 < 0 ? f64 : y_f64 != 0;
  if (f64 && yd)
    hipLaunchKernelGGL((reduce_partials_kernel<double, double>), dim3(blocks), dim3(threads), 0,
                       st, (const double*)part, nranges, r1, q, (double*)Y, Yd, flag);
  else if (f64)
    hipLaunchKernelGGL((reduce_partials_kernel<double, float>), dim3(blocks), dim3(threads), 0,
                       st, (const double*)part, nranges, r1, q, (float*)Y, Yd, flag);
  else if (!yd)
    hipLaunchKernelGGL((reduce_partials_kernel<float, float>), dim3(blocks), dim3(threads), 0,
                       st, (const float*)part, nranges, r1, q, (float*)Y, Yd, flag);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---- diagnostics ---------------------------------------------------------

__global__ void rng_words_kernel(uint32_t stream, uint64_t seed, uint64_t idx0, int64_t count,
                                 uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint4 w = stream_words(seed, stream, idx0 + (uint64_t)i, 0);
  out[4 * i + 0] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

__global__ void pi1_streams_kernel(uint64_t seed, uint32_t r1, int log2s, uint64_t j0,
                                   int64_t count, int32_t* bh, float* ch, int32_t* bi, float* ci,
                                   int8_t* sg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t j = j0 + (uint64_t)i;
  const uint64_t kH = h_position(j, log2s);
  uint32_t b0, w0, b1, w1;
  position_words(seed, 0, kH, r1, &b0, &w0);
  position_words(seed, 0, kH + (1ull << log2s), r1, &b1, &w1);
  bh[i] = (int32_t)b0;
  ch[i] = cauchy_from_word(w0);
  bi[i] = (int32_t)b1;
  ci[i] = cauchy_from_word(w1);
  const uint4 sw = stream_words(seed, kStreamSign, j >> 7, 0);
  sg[i] = (int8_t)sign_from_words(sw, j);
}

// Normalized FWHT of consecutive s-blocks, with the sketch's tile passes.
__global__ void __launch_bounds__(256) fwht_kernel(float* x, int64_t nblocks, int s, int log2s) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* tile = reinterpret_cast<float*>(smem_raw);
  const int chunk = s;
  const int TP = chunk + (chunk >> 4);
  const int64_t blk = blockIdx.x;
  if (blk >= nblocks) return;
  float* p = x + blk * s;
  for (int t = threadIdx.x; t < s; t += blockDim.x) tile[tpad(t)] = p[t];
  __syncthreads();
  fwht_tile<float>(tile, TP, 1, chunk, log2s);
  const float sc = 1.0f / sqrtf((float)s);
  for (int t = threadIdx.x; t < s; t += blockDim.x) p[t] = tile[tpad(t)] * sc;
}

hipError_t launch_rng_words(uint32_t stream, uint64_t seed, uint64_t idx0, int64_t count,
                            uint32_t* out, hipStream_t st) {
  const int threads = 256;
  hipLaunchKernelGGL(rng_words_kernel, dim3((unsigned)((count + threads - 1) / threads)),
                     dim3(threads), 0, st, stream, seed, idx0, count, out);
  return hipGetLastError();
}

hipError_t launch_pi1_streams(uint64_t seed, uint32_t r1, int log2s, uint64_t j0, int64_t count,
                              int32_t* bh, float* ch, int32_t* bi, float* ci, int8_t* sg,
                              hipStream_t st) {
  const int threads = 256;
  hipLaunchKernelGGL(pi1_streams_kernel, dim3((unsigned)((count + threads - 1) / threads)),
                     dim3(threads), 0, st, seed, r1, log2s, j0, count, bh, ch, bi, ci, sg);
  return hipGetLastError();
}

hipError_t launch_fwht(float* x, int64_t nblocks, int s, int log2s, hipStream_t st) {
  const size_t lds = (size_t)(s + (s >> 4)) * sizeof(float);
  hipLaunchKernelGGL(fwht_kernel, dim3((unsigned)nblocks), dim3(256), lds, st, x, nblocks, s,
                     log2s);
  return hipGetLastError();
}

}  // namespace fctl1
