// Walsh-Hadamard butterflies on data held across the 64 lanes of a wave
// (gfx950): register stages, DPP moves inside rows of 16 lanes, and the
// permlane swaps that trade a lane bit for a register bit.
//
// Layout used by the pass-1 kernels: a lane holds 16 values v[r],
// r = i + 4 k (i, k < 4), of a 1024-row span; value (lane l, register r) is
// row t = i + 4 l + 256 k, so row bits 0-1 are register bits 0-1, row bits
// 2-7 are lane bits 0-5 and row bits 8-9 are register bits 2-3.  The
// normalized transform H_s (Sylvester order, section "FCT1 Construction")
// of every s-block of the span needs butterflies over row bits below log2 s.
#pragma once
#include <hip/hip_runtime.h>

namespace fctl1 {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// v of the lane whose L differs in bit B (L = lane % 16: DPP within a row of
// 16 lanes).  Bit 0: quad_perm [1,0,3,2]; bit 1: quad_perm [2,3,0,1]; bit 2:
// row_half_mirror (L ^ 7) then quad_perm [3,2,1,0] (^ 3); bit 3: row_ror:8.
template <int B>
__device__ __forceinline__ float lane_xor(float v) {
  if constexpr (B == 0) return dpp_f<0xB1>(v);
  else if constexpr (B == 1) return dpp_f<0x4E>(v);
  else if constexpr (B == 2) return dpp_f<0x1B>(dpp_f<0x141>(v));
  else return dpp_f<0x128>(v);
}

// butterflies along bit B of L: the lower lane keeps x + y, the upper one
// x - y, as p + (+-1) v with one rounding, like x + y and x - y
template <int B>
__device__ __forceinline__ void lane_stage(float (&v)[16], int L) {
  const float sg = ((L >> B) & 1) ? -1.0f : 1.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float p = lane_xor<B>(v[r]);
    v[r] = fmaf(sg, v[r], p);
  }
}

__device__ __forceinline__ void bfly(float& a, float& b) {
  const float x = a, y = b;
  a = x + y;
  b = x - y;
}

// butterflies along register-index bit `rb` (0..3) of a 16-value vector
__device__ __forceinline__ void reg_stage(float (&v)[16], int rb) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if (!((r >> rb) & 1)) {
      switch (rb) {
        case 0: bfly(v[r], v[r + 1]); break;
        case 1: bfly(v[r], v[r + 2]); break;
        case 2: bfly(v[r], v[r + 4]); break;
        default: bfly(v[r], v[r + 8]); break;
      }
    }
}

// v_permlane16_swap on the register pairs (r, r + 4): the odd 16-lane rows of
// v[r] trade places with the even rows of v[r + 4].  Afterwards register bit
// 2 holds what lane bit 4 held and lane bit 4 what register bit 2 held, so
// the butterflies over the former lane bit are register butterflies.
__device__ __forceinline__ void swap16_stage(float (&v)[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if (!((r >> 2) & 1)) {
      const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[r]),
                                                      __float_as_uint(v[r + 4]), false, false);
      const float a = __uint_as_float(p[0]), b = __uint_as_float(p[1]);
      v[r] = a + b;
      v[r + 4] = a - b;
    }
}

// the same with v_permlane32_swap (halves of 32 lanes): lane bit 5 and
// register bit 3 trade places, then butterflies over register bit 3
__device__ __forceinline__ void swap32_stage(float (&v)[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    if (!((r >> 3) & 1)) {
      const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[r]),
                                                      __float_as_uint(v[r + 8]), false, false);
      const float a = __uint_as_float(p[0]), b = __uint_as_float(p[1]);
      v[r] = a + b;
      v[r + 8] = a - b;
    }
}

// Unnormalized H_s of every s-block of a 1024-row span in the layout above
// (s <= 1024; wave-uniform log2s).  Row bits 0, 1, 8, 9 are butterflied in
// registers, row bits 2-5 through DPP, and row bits 6 and 7 after the
// permlane swaps move them into register bits 2 and 3.  On return value
// (l, r) holds row t_out(l, r): row bits 0-5 as on entry, and when s > 64
// (s > 128) row bit 6 (7) comes from register bit 2 (3) and row bit 8 (9)
// from lane bit 4 (5).  Swapped bits above log2 s only move whole blocks.
__device__ __forceinline__ void fwht_span1024(float (&v)[16], int L, int log2s) {
  if (log2s > 0) reg_stage(v, 0);
  if (log2s > 1) reg_stage(v, 1);
  if (log2s > 8) reg_stage(v, 2);
  if (log2s > 9) reg_stage(v, 3);
  if (log2s > 2) lane_stage<0>(v, L);
  if (log2s > 3) lane_stage<1>(v, L);
  if (log2s > 4) lane_stage<2>(v, L);
  if (log2s > 5) lane_stage<3>(v, L);
  if (log2s > 6) swap16_stage(v);
  if (log2s > 7) swap32_stage(v);
}

// The same transform with log2 s fixed at compile time and the DPP stages in
// one instruction each: w <- w + sg * w_partner (v_fmac with the partner's
// value read through DPP), sg = +1 in the lower lane and -1 in the upper one.
// The lower lane gets x + y; the upper one gets y - x = -(x - y), so after
// the stages over lane bits 0..m-1 a lane holds its outputs times
// (-1)^popcount(L & (2^m - 1)) (span_sign).  Both lanes of a pair carry the
// same sign before the stage (they differ only in the stage's bit), the
// register stages and the permlane swaps keep the sign of the row of 16 they
// work in, so the factor is per lane and the caller folds it into its
// scaling.
template <int B>
__device__ __forceinline__ void lane_stage_signed(float (&v)[16], float sg) {
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = fmaf(lane_xor<B>(v[r]), sg, v[r]);
}

template <int LOG2S>
__device__ __forceinline__ void fwht_span1024_t(float (&v)[16], int L) {
  if constexpr (LOG2S > 0) reg_stage(v, 0);
  if constexpr (LOG2S > 1) reg_stage(v, 1);
  if constexpr (LOG2S > 8) reg_stage(v, 2);
  if constexpr (LOG2S > 9) reg_stage(v, 3);
  if constexpr (LOG2S > 2) lane_stage_signed<0>(v, (L & 1) ? -1.0f : 1.0f);
  if constexpr (LOG2S > 3) lane_stage_signed<1>(v, (L & 2) ? -1.0f : 1.0f);
  if constexpr (LOG2S > 4) lane_stage_signed<2>(v, (L & 4) ? -1.0f : 1.0f);
  if constexpr (LOG2S > 5) lane_stage_signed<3>(v, (L & 8) ? -1.0f : 1.0f);
  if constexpr (LOG2S > 6) swap16_stage(v);
  if constexpr (LOG2S > 7) swap32_stage(v);
}

// Signed DPP butterflies in one v_fmac_f32_dpp per value: v <- dpp(v) sg + v,
// dpp(v) the partner lane's value under the stage's DPP control.  The
// compiler does not see the DPP inside the asm, so the block keeps its own
// wait states: a DPP read needs two after a VALU write of the register and
// five after a scalar write of EXEC, hence the s_nop 4 in front; the
// instructions of a block read and write distinct registers, and the
// closing s_nop 1 covers whatever reads the results next.
#define FCT_FMAC_DPP(i, ctrl) "v_fmac_f32_dpp %" #i ", %" #i ", %16 " ctrl " row_mask:0xf bank_mask:0xf\n\t"
#define FCT_FMAC_DPP_BLOCK(ctrl)                                                                  \
  asm("s_nop 4\n\t" FCT_FMAC_DPP(0, ctrl) FCT_FMAC_DPP(1, ctrl) FCT_FMAC_DPP(2, ctrl)           \
          FCT_FMAC_DPP(3, ctrl) FCT_FMAC_DPP(4, ctrl) FCT_FMAC_DPP(5, ctrl) FCT_FMAC_DPP(6, ctrl) \
              FCT_FMAC_DPP(7, ctrl) FCT_FMAC_DPP(8, ctrl) FCT_FMAC_DPP(9, ctrl)                   \
                  FCT_FMAC_DPP(10, ctrl) FCT_FMAC_DPP(11, ctrl) FCT_FMAC_DPP(12, ctrl)            \
                      FCT_FMAC_DPP(13, ctrl) FCT_FMAC_DPP(14, ctrl) FCT_FMAC_DPP(15, ctrl)        \
      "s_nop 1"                                                                                   \
      : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]),    \
        "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]), "+v"(v[12]), "+v"(v[13]), \
        "+v"(v[14]), "+v"(v[15])                                                                \
      : "v"(sg))

// partner lanes L ^ 1, L ^ 2 (quad_perm), L ^ 7 (row_half_mirror), L ^ 8 (row_ror:8)
template <int P>
__device__ __forceinline__ void lane_stage_fmac(float (&v)[16], float sg) {
  if constexpr (P == 1) FCT_FMAC_DPP_BLOCK("quad_perm:[1,0,3,2]");
  else if constexpr (P == 2) FCT_FMAC_DPP_BLOCK("quad_perm:[2,3,0,1]");
  else if constexpr (P == 7) FCT_FMAC_DPP_BLOCK("row_half_mirror");
  else {
    static_assert(P == 8, "partner offsets of the DPP stages");
    FCT_FMAC_DPP_BLOCK("row_ror:8");
  }
}

// The transform of fwht_span1024_t with every lane stage one DPP instruction
// per value.  Lane bit 2 has no single-instruction partner L ^ 4, so for
// s >= 32 the stages over lane bits 0-2 run along L ^ 1, L ^ 2 and L ^ 7 in
// the coordinates c0 = l0 ^ l2, c1 = l1 ^ l2, c2 = l2 of L (l_i its bits):
// those partners differ in exactly one coordinate, so the three stages are
// the size-8 transform over (c0, c1, c2), each stage's sign taken from its
// own coordinate.  In lane coordinates the output of lane L is then the one
// of index pi(L & 7) | (L & 8) (pi: see span_row_out_dpp)
// with the sign span_sign(L, log2s), the same per-lane sign as in the
// standard order.
template <int LOG2S>
__device__ __forceinline__ void fwht_span1024_dpp(float (&v)[16], int L) {
  if constexpr (LOG2S > 0) reg_stage(v, 0);
  if constexpr (LOG2S > 1) reg_stage(v, 1);
  if constexpr (LOG2S > 8) reg_stage(v, 2);
  if constexpr (LOG2S > 9) reg_stage(v, 3);
  const int l0 = L & 1, l1 = (L >> 1) & 1, l2 = (L >> 2) & 1;
  if constexpr (LOG2S > 4) {
    lane_stage_fmac<1>(v, (l0 ^ l2) ? -1.0f : 1.0f);
    lane_stage_fmac<2>(v, (l1 ^ l2) ? -1.0f : 1.0f);
    lane_stage_fmac<7>(v, l2 ? -1.0f : 1.0f);
  } else {
    if constexpr (LOG2S > 2) lane_stage_fmac<1>(v, l0 ? -1.0f : 1.0f);
    if constexpr (LOG2S > 3) lane_stage_fmac<2>(v, l1 ? -1.0f : 1.0f);
  }
  if constexpr (LOG2S > 5) lane_stage_fmac<8>(v, (L & 8) ? -1.0f : 1.0f);
  if constexpr (LOG2S > 6) swap16_stage(v);
  if constexpr (LOG2S > 7) swap32_stage(v);
}

// the per-lane sign fwht_span1024_t leaves on its outputs
__device__ __forceinline__ float span_sign(int L, int log2s) {
  const int m = log2s > 6 ? 4 : (log2s > 2 ? log2s - 2 : 0);
  return (__builtin_popcount(L & ((1 << m) - 1)) & 1) ? -1.0f : 1.0f;
}

// Row within the 1024-row span of value (lane, register r) after
// fwht_span1024 with the given log2s.
__device__ __forceinline__ int span_row_out(int lane, int r, int log2s) {
  const int i = r & 3, k0 = (r >> 2) & 1, k1 = (r >> 3) & 1;
  const int l4 = (lane >> 4) & 1, l5 = (lane >> 5) & 1;
  const bool s6 = log2s > 6, s7 = log2s > 7;
  const int b6 = s6 ? k0 : l4, b8 = s6 ? l4 : k0;
  const int b7 = s7 ? k1 : l5, b9 = s7 ? l5 : k1;
  return i + 4 * (lane & 15) + 64 * b6 + 128 * b7 + 256 * b8 + 512 * b9;
}

// Row within the 1024-row span of value (lane, register r) after
// fwht_span1024_dpp<log2s>: span_row_out of the lane whose low three bits
// are pi(lane & 7), pi(k) = (k0 ^ k2) | (k1 ^ k2) << 1 | (k0 ^ k1 ^ k2) << 2,
// when log2s >= 5.
__device__ __forceinline__ int span_row_out_dpp(int lane, int r, int log2s) {
  if (log2s > 4) {
    const int k0 = lane & 1, k1 = (lane >> 1) & 1, k2 = (lane >> 2) & 1;
    lane = (lane & ~7) | (k0 ^ k2) | ((k1 ^ k2) << 1) | ((k0 ^ k1 ^ k2) << 2);
  }
  return span_row_out(lane, r, log2s);
}

}  // namespace fctl1
