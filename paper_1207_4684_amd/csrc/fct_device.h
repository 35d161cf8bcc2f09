// Device-side building blocks shared by the fctl1 kernels (gfx950, wave64).
//
// Random streams: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a
// 128-bit counter, a 64-bit key, ten rounds of two 32x32->64-bit products
// with the multipliers 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule
// 0x9E3779B9 / 0xBB67AE85.  Stream layout (key = seed, counter =
// (idx lo, idx hi, stream, instance)):
//   stream 0: idx = k >> 1 for stacked position k (FCT1: column k of B and
//             diagonal entry k of C): words (0, 1) -> bucket and Cauchy of the
//             even position, words (2, 3) -> those of the odd one.  Row j of
//             block b = j / s sits at k = 2 s b + (j mod s) (H-half) and
//             k + s (I-half);
//   stream 1: idx = j >> 7, bit j & 31 of word (j >> 5) & 3 -> sign D(j);
//   stream 2: idx = a * r2 + c, word 0 -> Cauchy Pi2[a][c] (words 0 and 1 ->
//             Gaussian Pi2[a][c] for the optimized regression);
//   stream 3: idx = i >> 2, word i & 3 -> uniform deciding row i (instance
//             k: the k-th of several draws from one sampling pass);
//   stream 4: idx = j >> 2, word j & 3 -> uniform of sample j of a draw with
//             replacement (instance k: the k-th draw);
//   stream 5: idx = g >> 2, g = beta s + k, word g & 3 -> the row of block
//             beta that sample k of FCT2's G takes;
//   stream 6: idx = g >> 2, g = i 2^40 + m, word g & 3 -> Cauchy C[i, m] of
//             FCT2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fctl1 {

enum : uint32_t {
  kStreamPi1 = 0,
  kStreamSign = 1,
  kStreamPi2 = 2,
  kStreamSample = 3,
  kStreamReplace = 4,
  kStreamFct2Rows = 5,
  kStreamFct2Cauchy = 6
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96: odd parity of the inputs)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                   xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 stream_words(uint64_t seed, uint32_t stream, uint64_t idx,
                                              uint32_t instance) {
  return philox4x32_10(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), stream, instance),
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Uniform bucket in [0, r1): floor(w * r1 / 2^32).
__device__ __forceinline__ uint32_t bucket_from_word(uint32_t w, uint32_t r1) {
  return __umulhi(w, r1);
}

// Standard Cauchy variate from a 32-bit word, FP32: the inverse CDF
// tan(pi (u - 1/2)) with u = (w + 1/2) / 2^32, evaluated without
// cancellation.  With m = min(w, 2^32 - 1 - w) the value is -/+ cot(pi v),
// v = (m + 1/2) / 2^32 in (0, 1/2) (minus for w < 2^31).  The argument is
// reduced to x = pi v' in (0, pi/4]: for v < 1/4, cot(pi v) = 1 / tan x with
// v' = v; otherwise cot(pi v) = tan(pi (1/2 - v)) = tan x with v' = 1/2 - v,
// whose numerator 2^31 - 1 - m + 1/2 is formed exactly in integers.  tan x is
// x P(x^2), P of degree 7 fitted to tan(x)/x on (0, pi/4] by least squares
// with Lawson's reweighting toward the minimax relative error (1.2e-9 in
// FP64, 4.6e-9 with the coefficients rounded to FP32); the argument is formed
// from an exact 22-bit/8-bit split of the integer numerator and a two-term
// FP32 split of pi 2^-32; the reciprocal is the hardware one refined by one
// Newton step.  Within about 3 FP32 ulp of the exact value.
__device__ __forceinline__ float cauchy_from_word(uint32_t w) {
  const bool neg = w < 0x80000000u;
  const uint32_t m = neg ? w : ~w;                   // < 2^31
  const bool lower = m < 0x40000000u;                // v < 1/4
  const uint32_t mr = lower ? m : (0x7FFFFFFFu - m); // < 2^30
  const float hi = (float)(mr >> 8) * 256.0f;        // exact
  const float lo = (float)(mr & 0xFFu) + 0.5f;       // exact
  const float K1 = 0x1.921fb6p-31f;                  // pi * 2^-32, FP32 head
  const float K2 = -0x1.777a5cp-56f;                 // remainder, FP32 tail
  const float x = fmaf(hi, K1, fmaf(hi, K2, lo * K1));
  const float u = x * x;
  float p = 0x1.21cebcp-8f;
  p = fmaf(u, p, -0x1.0785dap-16f);
  p = fmaf(u, p, 0x1.663ab0p-7f);
  p = fmaf(u, p, 0x1.5bf394p-6f);
  p = fmaf(u, p, 0x1.baf340p-5f);
  p = fmaf(u, p, 0x1.110cd0p-3f);
  p = fmaf(u, p, 0x1.555566p-2f);
  p = fmaf(u, p, 1.0f);
  const float t = x * p;  // tan x, in [3.7e-10, 1]: normal, no overflow of 1 / t
  // reciprocal: v_rcp_f32 (about 1 ulp) and one Newton step r (2 - t r)
  float r = __builtin_amdgcn_rcpf(t);
  r = fmaf(fmaf(-t, r, 1.0f), r, r);
  const float c = lower ? r : t;
  return neg ? -c : c;
}

// FP64 Cauchy for Pi2 (a few hundred values per regression).
__device__ __forceinline__ double cauchy_from_word_f64(uint32_t w) {
  const bool neg = w < 0x80000000u;
  const uint32_t m = neg ? w : ~w;
  const double v = ((double)m + 0.5) * 0x1p-32;
  const double c = 1.0 / tan(3.141592653589793 * v);
  return neg ? -c : c;
}

// FP64 standard Gaussian for the optimized regression's Pi2, from two words
// of one stream-2 call by the Box-Muller transform: with u = (w + 1/2) / 2^32,
// sqrt(-2 ln u1) cos(2 pi u2) is N(0, 1) for independent uniforms u1, u2.
__device__ __forceinline__ double gaussian_from_words_f64(uint32_t w0, uint32_t w1) {
  const double u1 = ((double)w0 + 0.5) * 0x1p-32;
  const double u2 = ((double)w1 + 0.5) * 0x1p-32;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Stacked position of the H-half copy of padded row j (the I-half is + s).
__device__ __forceinline__ uint64_t h_position(uint64_t j, int log2s) {
  return ((j >> log2s) << (log2s + 1)) + (j & ((1ull << log2s) - 1));
}

// (bucket, Cauchy word) of stacked position k (stream 0).
__device__ __forceinline__ void position_words(uint64_t seed, uint32_t instance, uint64_t k,
                                               uint32_t r1, uint32_t* bucket, uint32_t* cw) {
  const uint4 w = stream_words(seed, kStreamPi1, k >> 1, instance);
  const bool odd = k & 1;
  *bucket = bucket_from_word(odd ? w.z : w.x, r1);
  *cw = odd ? w.w : w.y;
}

// sign D(j) of stream 1 as +1 / -1
__device__ __forceinline__ float sign_from_words(uint4 wv, uint64_t j) {
  const uint32_t sel = (uint32_t)(j >> 5) & 3u;
  const uint32_t word = sel == 0 ? wv.x : sel == 1 ? wv.y : sel == 2 ? wv.z : wv.w;
  return ((word >> (j & 31u)) & 1u) ? -1.0f : 1.0f;
}

// Sum over the 64 lanes of a wave, the same value in every lane; every lane
// must be active.  Within each row of 16 lanes: DPP xor 1 and xor 2
// (quad_perm [1,0,3,2], [2,3,0,1]), then the half-row mirror (lane i with
// 7 - i: the other quad) and the row mirror (i with 15 - i: the other half);
// the four row sums are read as scalars and added in a fixed order.  About a
// tenth of the latency of six cross-lane shuffles through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

template <typename T> struct FmaT;
template <> struct FmaT<float> {
  static __device__ __forceinline__ float fma(float a, float b, float c) { return fmaf(a, b, c); }
};
template <> struct FmaT<double> {
  static __device__ __forceinline__ double fma(double a, double b, double c) { return ::fma(a, b, c); }
};

}  // namespace fctl1
