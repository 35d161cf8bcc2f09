// Pass 2: lambda_i = median_j |(X M)_ij| with M = R^-1 Pi2 (regression figure
// steps 4-5; the proof's running-time paragraph forms R^-1 Pi2 first and then
// X (R^-1 Pi2), O(n q r2), and takes each median of r2 values in O(r2)).
//
// One thread per row: the q values of the row are streamed column by column
// (coalesced across the wavefront, column-major X), the r2 dot products are
// accumulated in registers against M held in scalar registers (M is uniform,
// stored q x R2P with zero padding), the |.| values are sorted by a bitonic
// network and the median (mean of the two middle values for even r2) is
// stored.  Each workgroup also emits its FP64 sum of lambda, combined later in
// a fixed order.
#include "fct_device.h"
#include "fct_kernels.h"

#include <cstdlib>

namespace fctl1 {

static constexpr int kP2Threads = 256;

template <typename TX> struct Load;
template <> struct Load<float> {
  typedef float A;
  static __device__ __forceinline__ float get(const void* p, int64_t i) {
    return reinterpret_cast<const float*>(p)[i];
  }
};
template <> struct Load<double> {
  typedef double A;
  static __device__ __forceinline__ double get(const void* p, int64_t i) {
    return reinterpret_cast<const double*>(p)[i];
  }
};
struct Bf16 {};
template <> struct Load<Bf16> {
  typedef float A;
  static __device__ __forceinline__ float get(const void* p, int64_t i) {
    return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(p)[i] << 16);
  }
};

// compare-exchange as a min and a max (v_min / v_max: no condition masks);
// |.| values and the +inf padding are never NaN for finite data
template <typename TA>
__device__ __forceinline__ void cex(TA& a, TA& b) {
  const TA lo = fmin(a, b), hi = fmax(a, b);
  a = lo;
  b = hi;
}

template <typename TA, int N>
__device__ __forceinline__ void bitonic_sort(TA (&v)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          if ((i & k) == 0) cex(v[i], v[l]);
          else cex(v[l], v[i]);
        }
      }
    }
  }
}

// Sorts v[o .. o + 7] with the 19-comparator network of depth 6 (Knuth,
// TAOCP vol. 3, section 5.3.4).
template <int N>
__device__ __forceinline__ void sort8(float (&v)[N], int o) {
  cex(v[o + 0], v[o + 2]); cex(v[o + 1], v[o + 3]); cex(v[o + 4], v[o + 6]); cex(v[o + 5], v[o + 7]);
  cex(v[o + 0], v[o + 4]); cex(v[o + 1], v[o + 5]); cex(v[o + 2], v[o + 6]); cex(v[o + 3], v[o + 7]);
  cex(v[o + 0], v[o + 1]); cex(v[o + 2], v[o + 3]); cex(v[o + 4], v[o + 5]); cex(v[o + 6], v[o + 7]);
  cex(v[o + 2], v[o + 4]); cex(v[o + 3], v[o + 5]);
  cex(v[o + 1], v[o + 4]); cex(v[o + 3], v[o + 6]);
  cex(v[o + 1], v[o + 2]); cex(v[o + 3], v[o + 4]); cex(v[o + 5], v[o + 6]);
}

// Median of |v[0]|, ..., |v[r2 - 1]| (r2 <= R2P; the rest of v is ignored):
// the mean of the order statistics (r2 - 1) / 2 and r2 / 2 (0-based), as the
// oracle forms it.
// For r2 = 16 the two halves are sorted and the statistics 7 and 8 of their
// union are min_i max(a_(i-1), b_(7-i)) and min_i max(a_(i-1), b_(8-i)) over
// the splits i of the first 8 (9) values between the sorted halves a and b;
// otherwise a bitonic sort and a uniform register index.
template <int R2P>
__device__ __forceinline__ float median_of(float (&v)[R2P], int r2) {
  if (R2P == 16 && r2 == 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = fabsf(v[j]);
    sort8(v, 0);
    sort8(v, 8);
    const float* a = v;
    const float* b = v + 8;
    float lo = fmin(b[7], a[7]);
#pragma unroll
    for (int i = 1; i < 8; ++i) lo = fmin(lo, fmax(a[i - 1], b[7 - i]));
    float hi = fmax(a[0], b[7]);
#pragma unroll
    for (int i = 2; i < 9; ++i) hi = fmin(hi, fmax(a[i - 1], b[8 - i]));
    return 0.5f * (lo + hi);
  }
#pragma unroll
  for (int j = 0; j < R2P; ++j) v[j] = j < r2 ? fabsf(v[j]) : INFINITY;
  bitonic_sort<float, R2P>(v);
  typedef float fvec __attribute__((ext_vector_type(R2P)));
  fvec w;
#pragma unroll
  for (int j = 0; j < R2P; ++j) w[j] = v[j];
  return 0.5f * (w[(r2 - 1) >> 1] + w[r2 >> 1]);
}

__host__ __device__ int r2_padded(int r2) {
  int p = 4;
  while (p < r2) p <<= 1;
  return p;
}

template <typename TA>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

template <typename TX, int R2P>
__global__ void __launch_bounds__(kP2Threads) pass2_valu_kernel(Pass2Args a) {
  typedef typename Load<TX>::A TA;
  __shared__ double red[kP2Threads / 64];
  const TA* __restrict__ M = reinterpret_cast<const TA*>(a.M);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double lsum = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    TA acc[R2P];
#pragma unroll
    for (int j = 0; j < R2P; ++j) acc[j] = TA(0);
    for (int col = 0; col < a.q; ++col) {
      TA x = (col < a.d) ? Load<TX>::get(a.A, i + (int64_t)col * a.lda)
                         : -Load<TX>::get(a.b, i + (int64_t)(col - a.d) * a.ldb);
#pragma unroll
      for (int j = 0; j < R2P; ++j) acc[j] = FmaT<TA>::fma(x, M[col * R2P + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < R2P; ++j) acc[j] = (j < a.r2) ? fabs(acc[j]) : TA(INFINITY);
    bitonic_sort<TA, R2P>(acc);
    const int k1 = (a.r2 - 1) >> 1, k2 = a.r2 >> 1;
    TA m1 = acc[0], m2 = acc[0];
#pragma unroll
    for (int j = 1; j < R2P; ++j) {
      m1 = (j == k1) ? acc[j] : m1;
      m2 = (j == k2) ? acc[j] : m2;
    }
    const TA lam = TA(0.5) * (m1 + m2);
    a.lambda[i] = (float)lam;
    lsum += (double)(float)lam;
  }
  const double s = block_sum<TA>(lsum, red);
  if (threadIdx.x == 0) a.wg_sums[blockIdx.x] = s;
}

// MFMA form for FP32 and BF16 data.  Lambda^T = M^T X^T is formed on the
// matrix cores: A = M^T (16 r2-columns x K) is constant and held in registers,
// B = X^T (K x 16 rows) comes straight from the column-major X.  Each wave
// takes 64-row tiles; lane l loads rows 4 (l % 16) .. 4 (l % 16) + 3 of its
// columns in one vector load per column (all of a tile's loads are issued
// before the first product, so a wave keeps a whole tile in flight), and
// MFMA tile i of the four takes rows 4 n + i.  D holds, in lane l, register
// i, the value (tile row l % 16, r2-column 4 (l / 16) + i).  FP32 uses
// v_mfma_f32_16x16x4f32 (K = 4 per instruction), BF16 uses
// v_mfma_f32_16x16x16bf16_1k (K = 16, products exact, FP32 accumulation).
// D goes through LDS so that lane l then owns row l of the tile, takes |.|,
// sorts its r2 values and stores the median.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float f4_comp(const float4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// LDS rows of one wave: MFMA tile i (rows 4 n + i of the 64-row tile) is
// stored in its own block of 16 rows; blocks are 4 floats apart beyond a
// multiple of 64 banks so the lane-per-row reads do not collide.
template <int LS>
__device__ __forceinline__ float* p2_tile_rows(float* L, int i) { return L + i * (16 * LS + 4); }

// Loads of one 64-row tile for the MFMA forms: lane (n4, g) takes rows
// 64 tt + 4 n4 .. + 3 of column 4 ks + g (FP32, one float4 per column) or of
// columns 16 ks + 4 g + j (BF16, one 8-byte load per column); columns past q
// and rows past n read as zero, columns from d on (B) are negated.
template <int KS>
__device__ __forceinline__ void p2_load_f32(const float* __restrict__ A, const float* __restrict__ bv,
                                            int64_t lda, int64_t ldb, int d, int q, int64_t n,
                                            bool vec, int64_t tt, int n4, int g, float4 (&dst)[KS]) {
  const int64_t rb = (tt << 6) + 4 * n4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = 4 * ks + g;
    float4 x4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (c < q) {
      const float* col = c < d ? A + (int64_t)c * lda : bv + (int64_t)(c - d) * ldb;
      if (vec && rb + 3 < n) {
        x4 = *reinterpret_cast<const float4*>(col + rb);
      } else {
        if (rb < n) x4.x = col[rb];
        if (rb + 1 < n) x4.y = col[rb + 1];
        if (rb + 2 < n) x4.z = col[rb + 2];
        if (rb + 3 < n) x4.w = col[rb + 3];
      }
      if (c >= d) x4 = make_float4(-x4.x, -x4.y, -x4.z, -x4.w);
    }
    dst[ks] = x4;
  }
}

template <int KS>
__device__ __forceinline__ void p2_load_bf16(const uint16_t* __restrict__ A,
                                             const uint16_t* __restrict__ bv, int64_t lda,
                                             int64_t ldb, int d, int q, int64_t n, bool vec,
                                             int64_t tt, int n4, int g, uint2 (&dst)[KS][4]) {
  const int64_t rb = (tt << 6) + 4 * n4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 16 * ks + 4 * g + j;
      uint2 x4 = make_uint2(0u, 0u);
      if (c < q) {
        const uint16_t* col = c < d ? A + (int64_t)c * lda : bv + (int64_t)(c - d) * ldb;
        if (vec && rb + 3 < n) {
          x4 = *reinterpret_cast<const uint2*>(col + rb);
        } else {
          const uint32_t e0 = rb < n ? col[rb] : 0u, e1 = rb + 1 < n ? col[rb + 1] : 0u;
          const uint32_t e2 = rb + 2 < n ? col[rb + 2] : 0u, e3 = rb + 3 < n ? col[rb + 3] : 0u;
          x4 = make_uint2(e0 | (e1 << 16), e2 | (e3 << 16));
        }
        if (c >= d) x4 = make_uint2(x4.x ^ 0x80008000u, x4.y ^ 0x80008000u);
      }
      dst[ks][j] = x4;
    }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): a tile loaded
// on the guarded path is complete before the paths join, so the join does not
// make the prefetching path wait for its own loads of the next tile.
__device__ __forceinline__ void p2_wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The same loads for a whole tile of aligned columns (rows 64 tt .. 64 tt + 63
// inside X), issued without branches so that they can stay in flight while
// the previous tile is processed: columns past q load column q - 1, and
// p2_fix_* zeroes them and negates the columns of B once the data is needed.
template <int KS>
__device__ __forceinline__ void p2_issue_f32(const float* __restrict__ A, const float* __restrict__ bv,
                                             int64_t lda, int64_t ldb, int d, int q, int64_t tt,
                                             int n4, int g, float4 (&raw)[KS]) {
  const int64_t rb = (tt << 6) + 4 * n4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = min(4 * ks + g, q - 1);
    const float* col = c < d ? A + (int64_t)c * lda : bv + (int64_t)(c - d) * ldb;
    raw[ks] = *reinterpret_cast<const float4*>(col + rb);
  }
}

template <int KS>
__device__ __forceinline__ void p2_fix_f32(int d, int q, int g, const float4 (&raw)[KS],
                                           float4 (&xv)[KS]) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int c = 4 * ks + g;
    const float sg = c < d ? 1.0f : -1.0f;
    const float4 x = raw[ks];
    xv[ks] = c < q ? make_float4(sg * x.x, sg * x.y, sg * x.z, sg * x.w)
                   : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

template <int KS>
__device__ __forceinline__ void p2_issue_bf16(const uint16_t* __restrict__ A,
                                              const uint16_t* __restrict__ bv, int64_t lda,
                                              int64_t ldb, int d, int q, int64_t tt, int n4, int g,
                                              uint2 (&raw)[KS][4]) {
  const int64_t rb = (tt << 6) + 4 * n4;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = min(16 * ks + 4 * g + j, q - 1);
      const uint16_t* col = c < d ? A + (int64_t)c * lda : bv + (int64_t)(c - d) * ldb;
      raw[ks][j] = *reinterpret_cast<const uint2*>(col + rb);
    }
}

template <int KS>
__device__ __forceinline__ void p2_fix_bf16(int d, int q, int g, const uint2 (&raw)[KS][4],
                                            uint2 (&xv)[KS][4]) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 16 * ks + 4 * g + j;
      const uint32_t flip = c < d ? 0u : 0x80008000u;
      const uint2 x = raw[ks][j];
      xv[ks][j] = c < q ? make_uint2(x.x ^ flip, x.y ^ flip) : make_uint2(0u, 0u);
    }
}

// KS: K-steps of 4 columns compiled in (the smallest of 3, 5, 9, 17 that
// covers q; columns past q read as zero).
template <int MT, int KS>
__global__ void __launch_bounds__(kP2Threads) pass2_mfma_f32_kernel(Pass2Args a) {
  constexpr int R2P = 16 * MT, LS = R2P + 4;
  __shared__ __align__(16) float lds[kP2Threads / 64][64 * LS + 12];
  __shared__ double red[kP2Threads / 64];
  // the wave index is uniform: readfirstlane lets the tile loop and its choices stay scalar
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r2p = r2_padded(a.r2);
  const float* __restrict__ Mf = reinterpret_cast<const float*>(a.M);
  const float* __restrict__ A = reinterpret_cast<const float*>(a.A);
  const float* __restrict__ bv = reinterpret_cast<const float*>(a.b);
  const bool vec = (a.lda & 3) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(bv) & 15) == 0 && (a.q - a.d <= 1 || (a.ldb & 3) == 0);
  // A operand: M[k][m], k = 4 ks + lane / 16, m = lane % 16 + 16 mt
  float am[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + (lane >> 4), m = (lane & 15) + 16 * mt;
      am[mt][ks] = (k < a.q && m < r2p) ? Mf[k * r2p + m] : 0.0f;
    }
  p2_wait_loads();  // M is in registers before the tile loop (no load is pending across it)
  float* L = lds[wave];
  double lsum = 0.0;
  const int64_t ntiles = (a.n + 63) >> 6;
  const int64_t tstride = (int64_t)gridDim.x * (kP2Threads / 64);
  const int n4 = lane & 15, g = lane >> 4;
  // rows 64 t + 4 n4 .. + 3 of column 4 ks + g, one float4 per column; MFMA
  // tile i takes row 64 t + 4 n4 + i
  // a whole aligned tile's loads are issued before the previous tile's
  // products (wave-uniform choice), so a wave keeps two tiles in flight
  float4 raw[KS];
  int64_t t = (int64_t)blockIdx.x * (kP2Threads / 64) + wave;
  bool pre = vec && t < ntiles && ((t + 1) << 6) <= a.n;
  if (pre) p2_issue_f32<KS>(A, bv, a.lda, a.ldb, a.d, a.q, t, n4, g, raw);
  for (; t < ntiles; t += tstride) {
    const int64_t r0 = t << 6;
    float4 xv[KS];
    if (pre) {
      p2_fix_f32<KS>(a.d, a.q, g, raw, xv);
    } else {
      p2_load_f32<KS>(A, bv, a.lda, a.ldb, a.d, a.q, a.n, vec, t, n4, g, xv);
      p2_wait_loads();
    }
    const int64_t tn = t + tstride;
    pre = vec && tn < ntiles && ((tn + 1) << 6) <= a.n;
    if (pre) p2_issue_f32<KS>(A, bv, a.lda, a.ldb, a.d, a.q, tn, n4, g, raw);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float* Li = p2_tile_rows<LS>(L, i);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(am[mt][ks], f4_comp(xv[ks], i), acc, 0, 0, 0);
        *reinterpret_cast<f32x4*>(Li + n4 * LS + 16 * mt + 4 * g) = acc;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane = 4 n + i holds row r0 + lane
    const float* Lr = p2_tile_rows<LS>(L, lane & 3) + (lane >> 2) * LS;
    float v[R2P];
#pragma unroll
    for (int j = 0; j < R2P; j += 4) {
      const f32x4 q4 = *reinterpret_cast<const f32x4*>(Lr + j);
      v[j] = q4[0];
      v[j + 1] = q4[1];
      v[j + 2] = q4[2];
      v[j + 3] = q4[3];
    }
    const float lam = median_of<R2P>(v, a.r2);
    const int64_t row = r0 + lane;
    if (row < a.n) {
      a.lambda[row] = lam;
      lsum += (double)lam;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const double s = block_sum<double>(lsum, red);
  if (threadIdx.x == 0) a.wg_sums[blockIdx.x] = s;
}

// KS: K-steps of 16 columns compiled in (ceil(q / 16), at most 5).
template <int MT, int KS>
__global__ void __launch_bounds__(kP2Threads) pass2_mfma_bf16_kernel(Pass2Args a) {
  constexpr int R2P = 16 * MT, LS = R2P + 4;
  __shared__ __align__(16) float lds[kP2Threads / 64][64 * LS + 12];
  __shared__ double red[kP2Threads / 64];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r2p = r2_padded(a.r2);
  const uint16_t* __restrict__ A = reinterpret_cast<const uint16_t*>(a.A);
  const uint16_t* __restrict__ bv = reinterpret_cast<const uint16_t*>(a.b);
  const bool vec = (a.lda & 3) == 0 && (reinterpret_cast<uintptr_t>(A) & 7) == 0 &&
                   (reinterpret_cast<uintptr_t>(bv) & 7) == 0 && (a.q - a.d <= 1 || (a.ldb & 3) == 0);
  // A operand: M[k][m] as BF16, k = 16 ks + 4 (lane / 16) + j, m = lane % 16 + 16 mt
  s16x4 am[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * ks + 4 * (lane >> 4) + j, m = (lane & 15) + 16 * mt;
        am[mt][ks][j] = (k < a.q && m < r2p) ? (short)a.Mb[k * r2p + m] : (short)0;
      }
  p2_wait_loads();  // M is in registers before the tile loop (no load is pending across it)
  float* L = lds[wave];
  double lsum = 0.0;
  const int64_t ntiles = (a.n + 63) >> 6;
  const int64_t tstride = (int64_t)gridDim.x * (kP2Threads / 64);
  const int n4 = lane & 15, g = lane >> 4;
  // rows 64 t + 4 n4 .. + 3 of columns 16 ks + 4 g + j: one 8-byte load per
  // column; MFMA tile i takes row 64 t + 4 n4 + i
  // a whole aligned tile's loads are issued before the previous tile's
  // products (wave-uniform choice), so a wave keeps two tiles in flight
  uint2 raw[KS][4];
  int64_t t = (int64_t)blockIdx.x * (kP2Threads / 64) + wave;
  bool pre = vec && t < ntiles && ((t + 1) << 6) <= a.n;
  if (pre) p2_issue_bf16<KS>(A, bv, a.lda, a.ldb, a.d, a.q, t, n4, g, raw);
  for (; t < ntiles; t += tstride) {
    const int64_t r0 = t << 6;
    uint2 xc[KS][4];
    if (pre) {
      p2_fix_bf16<KS>(a.d, a.q, g, raw, xc);
    } else {
      p2_load_bf16<KS>(A, bv, a.lda, a.ldb, a.d, a.q, a.n, vec, t, n4, g, xc);
      p2_wait_loads();
    }
    const int64_t tn = t + tstride;
    pre = vec && tn < ntiles && ((tn + 1) << 6) <= a.n;
    if (pre) p2_issue_bf16<KS>(A, bv, a.lda, a.ldb, a.d, a.q, tn, n4, g, raw);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float* Li = p2_tile_rows<LS>(L, i);
      s16x4 xb[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t w = (i < 2) ? xc[ks][j].x : xc[ks][j].y;
          xb[ks][j] = (short)((i & 1) ? (w >> 16) : (w & 0xFFFFu));
        }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am[mt][ks], xb[ks], acc, 0, 0, 0);
        *reinterpret_cast<f32x4*>(Li + n4 * LS + 16 * mt + 4 * g) = acc;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float* Lr = p2_tile_rows<LS>(L, lane & 3) + (lane >> 2) * LS;
    float v[R2P];
#pragma unroll
    for (int j = 0; j < R2P; j += 4) {
      const f32x4 q4 = *reinterpret_cast<const f32x4*>(Lr + j);
      v[j] = q4[0];
      v[j + 1] = q4[1];
      v[j + 2] = q4[2];
      v[j + 3] = q4[3];
    }
    const float lam = median_of<R2P>(v, a.r2);
    const int64_t row = r0 + lane;
    if (row < a.n) {
      a.lambda[row] = lam;
      lsum += (double)lam;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const double s = block_sum<double>(lsum, red);
  if (threadIdx.x == 0) a.wg_sums[blockIdx.x] = s;
}

int pass2_grid(int64_t n, int kind, int cap_override) {
  if (kind != kPass2F64) {
    // MFMA forms: 64-row tiles per wave, grid-stride over the tiles
    int64_t cap = cap_override > 0 ? cap_override : 1024;
    int64_t want = (n + 255) / 256;
    if (want > cap) want = cap;
    return (int)(want < 1 ? 1 : want);
  }
  int64_t want = (n + kP2Threads - 1) / kP2Threads;
  if (want > 2048) want = 2048;
  return (int)(want < 1 ? 1 : want);
}

template <typename TX>
static hipError_t launch_pass2_t(const Pass2Args& a, int r2p, int grid, hipStream_t st) {
  switch (r2p) {
    case 4: hipLaunchKernelGGL((pass2_valu_kernel<TX, 4>), dim3(grid), dim3(kP2Threads), 0, st, a); break;
    case 8: hipLaunchKernelGGL((pass2_valu_kernel<TX, 8>), dim3(grid), dim3(kP2Threads), 0, st, a); break;
    case 16: hipLaunchKernelGGL((pass2_valu_kernel<TX, 16>), dim3(grid), dim3(kP2Threads), 0, st, a); break;
    case 32: hipLaunchKernelGGL((pass2_valu_kernel<TX, 32>), dim3(grid), dim3(kP2Threads), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


hipError_t launch_pass2(const Pass2Args& a, int kind, int grid, hipStream_t st) {
  const int r2p = r2_padded(a.r2);
  if (grid < 1) return hipErrorInvalidValue;
  if (kind == kPass2F64) return launch_pass2_t<double>(a, r2p, grid, st);
  if (a.q > 65 || a.r2 > 32) return hipErrorInvalidValue;
  if (kind == kPass2BF16) {
    const int ks = (a.q + 15) >> 4;
#define P2_BF16(MT, KS) hipLaunchKernelGGL((pass2_mfma_bf16_kernel<MT, KS>), dim3(grid), dim3(kP2Threads), 0, st, a)
    if (r2p <= 16) {
      switch (ks) {
        case 1: P2_BF16(1, 1); break;
        case 2: P2_BF16(1, 2); break;
        case 3: P2_BF16(1, 3); break;
        case 4: P2_BF16(1, 4); break;
        default: P2_BF16(1, 5); break;
      }
    } else {
      switch (ks) {
        case 1: P2_BF16(2, 1); break;
        case 2: P2_BF16(2, 2); break;
        case 3: P2_BF16(2, 3); break;
        case 4: P2_BF16(2, 4); break;
        default: P2_BF16(2, 5); break;
      }
    }
#undef P2_BF16
  } else {
    const int ks = (a.q + 3) >> 2;
#define P2_F32(MT, KS) hipLaunchKernelGGL((pass2_mfma_f32_kernel<MT, KS>), dim3(grid), dim3(kP2Threads), 0, st, a)
    if (r2p <= 16) {
      if (ks <= 3) P2_F32(1, 3);
      else if (ks <= 5) P2_F32(1, 5);
      else if (ks <= 9) P2_F32(1, 9);
      else P2_F32(1, 17);
    } else {
      if (ks <= 3) P2_F32(2, 3);
      else if (ks <= 5) P2_F32(2, 5);
      else if (ks <= 9) P2_F32(2, 9);
      else P2_F32(2, 17);
    }
#undef P2_F32
  }
  return hipGetLastError();
}

// out = sum of parts[0..count) in a fixed order (one workgroup).
__global__ void sum_fixed_kernel(const double* __restrict__ parts, int count, double* out) {
  __shared__ double red[256 / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) v += parts[i];
  const double s = block_sum<double>(v, red);
  if (threadIdx.x == 0) *out = s;
}

hipError_t launch_sum_fixed(const double* parts, int count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_fixed_kernel, dim3(1), dim3(256), 0, st, parts, count, out);
  return hipGetLastError();
}

}  // namespace fctl1
