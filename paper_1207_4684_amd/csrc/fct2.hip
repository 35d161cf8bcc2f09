// FCT2 (section "FCT2 Construction"): Pi1 = 8/r1 sqrt(pi t / (2 s)) C Hbar.
//
// Hbar is block-diagonal with n' / t copies of the s x t matrix
// G = sqrt(t/s) P H_t D: D the signs of stream 1 (indexed by global row, as
// for FCT1), H_t the normalized Hadamard matrix of order t in Sylvester order,
// P keeping s rows of t drawn uniformly with replacement (stream 5, sample
// g = beta s + k of global block beta takes row floor(w t / 2^32)).  C is an
// r1 x (n' s / t) matrix of standard Cauchy variates, C[i, m] from word
// g & 3 of stream 6 at idx g >> 2, g = i 2^40 + m.  Rows are zero-padded to
// n' = t ceil(n / t).
//
// Two kernels:
//  * fct2_fjlt_kernel -- one single-wave workgroup per block of t rows.  For
//    each column it applies D, takes the unnormalized FWHT of order t (the
//    register bits of the element index in registers, an LDS transpose, the
//    remaining lane bits in registers and the lowest ones across lanes) and
//    writes the s sampled outputs divided by sqrt(s) (= G z) in FP64 to Z,
//    row-major (n' s / t) x zq.  Streams X once: HBM-bound.
//  * fct2_cauchy_kernel -- the dense contraction Y = c C Z.  A thread owns
//    one row i of C and a chunk of m; C is never stored (one Philox call
//    gives C[i, m .. m + 3]); tiles of Z rows are staged in LDS and read as
//    wave-uniform broadcasts; FP64 accumulators.  Per-chunk partials are
//    reduced in a fixed order by launch_reduce_partials.  Bound by the
//    generation of C (VALU).
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

template <typename T, int LOG2T>
__global__ void __launch_bounds__(64) fct2_fjlt_kernel(Fct2Args a) {
  constexpr int TT = 1 << LOG2T;
  constexpr int P = TT / 64;       // values per lane
  constexpr int PAD = 64 / P;      // lanes sharing one register set after the transpose
  constexpr int ROW = 64 + PAD;    // padded LDS row of 64 elements
  __shared__ T buf[P * ROW];
  __shared__ uint32_t sw[TT / 32];
  __shared__ int32_t rows[kFct2MaxS];
  const int l = threadIdx.x;
  // blocks beta0 + blockIdx.x, + gridDim.x, ... (the grid may be capped to leave
  // room for a concurrent contraction)
  for (int64_t bb = blockIdx.x; bb < a.nbl; bb += gridDim.x) {
    __syncthreads();  // the previous block's reads of sw and rows are done
    const int64_t beta = a.beta0 + bb;
    const int64_t r0 = beta * TT;
    const uint64_t g0 = (uint64_t)(a.row0g + r0);

    // sign words of the block's rows (stream 1: bit j & 31 of word (j >> 5) & 3
    // of call j >> 7) and the s sampled rows (stream 5)
    for (int k = l; k < TT / 32; k += 64) {
      const uint64_t j = g0 + 32ull * (uint64_t)k;
      const uint4 w = stream_words(a.seed, kStreamSign, j >> 7, a.instance);
      const uint32_t sel = (uint32_t)(j >> 5) & 3u;
      sw[k] = sel == 0 ? w.x : sel == 1 ? w.y : sel == 2 ? w.z : w.w;
    }
    const uint64_t gbeta = (uint64_t)(a.row0g / TT + beta);
    for (int k = l; k < a.s; k += 64) {
      const uint64_t g = gbeta * (uint64_t)a.s + (uint64_t)k;
      const uint4 w = stream_words(a.seed, kStreamFct2Rows, g >> 2, a.instance);
      const uint32_t sel = (uint32_t)g & 3u;
      const uint32_t wd = sel == 0 ? w.x : sel == 1 ? w.y : sel == 2 ? w.z : w.w;
      rows[k] = (int32_t)(wd >> (32 - LOG2T));  // floor(w t / 2^32)
    }
    __syncthreads();
    // bit m: D is -1 at element m * 64 + l
    uint64_t smask = 0;
#pragma unroll
    for (int m = 0; m < P; ++m)
      smask |= (uint64_t)((sw[2 * m + (l >> 5)] >> (l & 31)) & 1u) << m;

    const int mm = l / PAD, ll = l % PAD;  // transposed role of this lane
    const double zscale = 1.0 / sqrt((double)a.s);
    for (int j = 0; j < a.q; ++j) {
      const bool negcol = j >= a.d;  // X = [A, -b]
      const T* col = negcol ? (const T*)a.b : (const T*)a.A + (size_t)j * a.lda;
      T v[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const int64_t row = r0 + m * 64 + l;
        const T x = row < a.n ? col[row] : T(0);
        v[m] = (((smask >> m) & 1) != 0) != negcol ? -x : x;
      }
      // element bits 6 .. LOG2T-1 (register index m)
#pragma unroll
      for (int h = 1; h < P; h <<= 1)
#pragma unroll
        for (int m = 0; m < P; ++m)
          if (!(m & h)) {
            const T u = v[m], w = v[m + h];
            v[m] = u + w;
            v[m + h] = u - w;
          }
      // element e lives at (e >> 6) * ROW + (e & 63)
#pragma unroll
      for (int m = 0; m < P; ++m) buf[m * ROW + l] = v[m];
      __syncthreads();
      // this lane now holds elements mm * 64 + lh * PAD + ll, lh < P
#pragma unroll
      for (int lh = 0; lh < P; ++lh) v[lh] = buf[mm * ROW + lh * PAD + ll];
      // element bits log2(PAD) .. 5 (register index lh)
#pragma unroll
      for (int h = 1; h < P; h <<= 1)
#pragma unroll
        for (int m = 0; m < P; ++m)
          if (!(m & h)) {
            const T u = v[m], w = v[m + h];
            v[m] = u + w;
            v[m + h] = u - w;
          }
      // element bits 0 .. log2(PAD) - 1 (lane bits of ll)
#pragma unroll
      for (int h = 1; h < PAD; h <<= 1)
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const T p = __shfl_xor(v[m], h, 64);
          v[m] = (l & h) ? p - v[m] : v[m] + p;
        }
      // each lane rewrites exactly the addresses it read
#pragma unroll
      for (int lh = 0; lh < P; ++lh) buf[mm * ROW + lh * PAD + ll] = v[lh];
      __syncthreads();
      for (int k = l; k < a.s; k += 64) {
        const int e = rows[k];
        a.Z[(size_t)(beta * a.s + k) * a.zq + j] = (double)buf[(e >> 6) * ROW + (e & 63)] * zscale;
      }
      __syncthreads();
    }
    // columns q .. zq-1 of Z are zero (the contraction reads whole slices)
    for (int k = l; k < a.s; k += 64)
      for (int j = a.q; j < a.zq; ++j) a.Z[(size_t)(beta * a.s + k) * a.zq + j] = 0.0;
  }
}

template <typename TC> __device__ __forceinline__ double fct2_cauchy(uint32_t w);
template <> __device__ __forceinline__ double fct2_cauchy<float>(uint32_t w) {
  return (double)cauchy_from_word(w);
}
template <> __device__ __forceinline__ double fct2_cauchy<double>(uint32_t w) {
  return cauchy_from_word_f64(w);
}

template <typename TC, int QC>
__global__ void __launch_bounds__(256) fct2_cauchy_kernel(Fct2Args a) {
  constexpr int MT = 64;  // rows of Z per LDS tile
  __shared__ double zt[MT * QC];
  const int i = blockIdx.y * 256 + threadIdx.x;
  const int64_t m0 = a.mbase + (int64_t)blockIdx.x * a.kc;
  const int64_t m1 = min(a.mend, m0 + a.kc);
  const double* __restrict__ zs = a.Z + (size_t)blockIdx.z * QC;
  const uint64_t ihi = (uint64_t)i << 38;  // (i 2^40 + m) >> 2 for m a multiple of 4
  double acc[QC];
#pragma unroll
  for (int jj = 0; jj < QC; ++jj) acc[jj] = 0.0;
  for (int64_t mt = m0; mt < m1; mt += MT) {
    const int rows = (int)min((int64_t)MT, m1 - mt);
    __syncthreads();  // the previous tile's reads are done
    for (int e = threadIdx.x; e < rows * QC; e += 256) {
      const int r = e / QC, jj = e - r * QC;
      zt[e] = zs[(size_t)(mt + r) * a.zq + jj];
    }
    __syncthreads();
    for (int r = 0; r < rows; r += 4) {  // mt and r are multiples of 4
      const uint4 w =
          stream_words(a.seed, kStreamFct2Cauchy, ihi | (uint64_t)((mt + r) >> 2), a.instance);
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = r + u < rows;
        const double cv = in ? fct2_cauchy<TC>(ws[u]) : 0.0;
        const double* z = zt + (in ? r + u : 0) * QC;  // wave-uniform: LDS broadcast
#pragma unroll
        for (int jj = 0; jj < QC; ++jj) acc[jj] = fma(cv, z[jj], acc[jj]);
      }
    }
  }
  if (i >= a.r1) return;
  double* out = a.partials + (size_t)(a.chunk0 + blockIdx.x) * a.r1 * a.q;
#pragma unroll
  for (int jj = 0; jj < QC; ++jj) {
    const int j = blockIdx.z * QC + jj;
    if (j < a.q) out[(size_t)j * a.r1 + i] = acc[jj] * a.scale;
  }
}

int fct2_slice_width(int q) { return q <= 8 ? 8 : q <= 17 ? 17 : 33; }

template <typename T>
static hipError_t launch_fjlt_t(const Fct2Args& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.fjlt_grid > 0 && a.fjlt_grid < a.nbl ? a.fjlt_grid : a.nbl));
  switch (a.log2t) {
    case 6: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 6>), grid, dim3(64), 0, st, a); break;
    case 7: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 7>), grid, dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 8>), grid, dim3(64), 0, st, a); break;
    case 9: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 9>), grid, dim3(64), 0, st, a); break;
    case 10: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 10>), grid, dim3(64), 0, st, a); break;
    case 11: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 11>), grid, dim3(64), 0, st, a); break;
    case 12: hipLaunchKernelGGL((fct2_fjlt_kernel<T, 12>), grid, dim3(64), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TC>
static hipError_t launch_cauchy_t(const Fct2Args& a, hipStream_t st) {
  const int qc = fct2_slice_width(a.q);
  const dim3 grid((unsigned)a.nchunks, (unsigned)((a.r1 + 255) / 256), (unsigned)(a.zq / qc));
  switch (qc) {
    case 8: hipLaunchKernelGGL((fct2_cauchy_kernel<TC, 8>), grid, dim3(256), 0, st, a); break;
    case 17: hipLaunchKernelGGL((fct2_cauchy_kernel<TC, 17>), grid, dim3(256), 0, st, a); break;
    case 33: hipLaunchKernelGGL((fct2_cauchy_kernel<TC, 33>), grid, dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fct2_fjlt(const Fct2Args& a, bool f64, hipStream_t st) {
  if (a.s < 1 || a.s > kFct2MaxS || a.s > (1 << a.log2t) || a.nbl < 1 || a.beta0 < 0 ||
      a.beta0 + a.nbl > a.nb || a.nb > 0x7FFFFFFF)
    return hipErrorInvalidValue;
  return f64 ? launch_fjlt_t<double>(a, st) : launch_fjlt_t<float>(a, st);
}

hipError_t launch_fct2_cauchy(const Fct2Args& a, bool f64, hipStream_t st) {
  if (a.kc < 4 || (a.kc & 3) || a.nchunks < 1 || (a.mbase & 3) || a.mbase < 0 ||
      a.mend > a.K || a.mbase + (int64_t)a.nchunks * a.kc < a.mend || a.chunk0 < 0 ||
      a.zq % fct2_slice_width(a.q) != 0)
    return hipErrorInvalidValue;
  return f64 ? launch_cauchy_t<double>(a, st) : launch_cauchy_t<float>(a, st);
}

}  // namespace fctl1
