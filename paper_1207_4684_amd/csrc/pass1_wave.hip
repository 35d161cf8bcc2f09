// Pass 1, wave-level form for FP32 data and s <= 2048: Y = Pi1 X with
// Pi1 = 4 B C H~ (section "FCT1 Construction"; n/s Hadamard transforms of
// size s, a diagonal Cauchy scaling and a hash scatter with 2n non-zeros).
//
// The random part of Pi1 (bucket and Cauchy of both stacked copies of every
// row) does not depend on X.  pi1_table_kernel draws it once per sketch into
// a table of 12 bytes per row (one Philox call per pair of stacked
// positions), so the column slices below read it instead of drawing it again.
//
// A workgroup of 8 waves owns a range of rows and a slice of c columns of
// X = [A, -b], with a private FP64 accumulator in LDS of r1 rows at a stride
// of pass1_acc_stride(c) doubles (FP64 LDS atomic adds: on gfx950 they
// sustain ~9x the rate of FP32 LDS atomic adds, and the sums are FP64).  Its
// waves take 256-row tiles:
//   1. the tile's table entries, 4 rows per lane (loaded one tile ahead), go
//      to the wave's table in LDS as (bucket * stride, Cauchy), shared by every
//      column;
//   2. the slice's columns are processed 4 at a time, 16 lanes per column; a
//      lane holds 16 rows {4L + i + 64k} of its column (float4 loads, the
//      next group's loads issued before the current group is processed);
//   3. the sign D(j) is applied, the I-half copies are added into their
//      buckets (LDS atomics), the Walsh-Hadamard butterflies over the row
//      bits held in registers (0, 1, 6, 7) are done in place, those over row
//      bits 2-5 (the lane index within 16) pair lanes through DPP moves, and
//      the H-half copies are added into their buckets.  No LDS beyond the
//      accumulator and the per-wave tables is touched, which leaves room
//      for wider column slices.
// pass1_wave_kernel (s <= 256): a 256-row tile holds whole blocks, each wave
// streams its own contiguous eighth of the range and never waits for the
// others, and it draws the signs of D itself (a Philox call per 128 rows).
// pass1_block_kernel (256 < s <= 2048): the workgroup walks its range in
// steps of 8 tiles, wave w taking tile w, so a block spans s / 256
// neighbouring waves; row bits 8-10 are the wave index and their butterflies
// pair the waves through an LDS exchange buffer (8 of a lane's 16 values at a
// time) at workgroup barriers.  Its signs come with the table (bit 15 of a
// row's key), so it keeps no sign words.  Either way the accumulator is
// written once per workgroup and the partials are summed in a fixed order by
// the reduction kernel.
#include "fct_device.h"
#include "fct_kernels.h"
#include "wave_fwht.h"

namespace fctl1 {

namespace {

constexpr int kTile = 256;
constexpr int kWaves = 8;
constexpr int kXch = 8 * 64;            // floats per wave in the cross-wave exchange (s > 256):
                                        // 8 of a lane's 16 values at a time
constexpr int kSignRows = 4096;         // rows covered by one refresh of sign words (s <= 256)

struct WaveTab {
  uint2 entH[kTile];                    // {bucket * stride, bits of 4 C / sqrt(s)} of the H-half copy
  uint2 entI[kTile];                    // {bucket * stride, bits of 4 C} of the I-half copy
};
struct WaveLds : WaveTab {
  uint32_t sgn[kSignRows / 32];         // sign words (s <= 256 form)
};

__device__ __forceinline__ void load_group(const Pass1Args& a, int c0, int cs, int64_t tile,
                                           int grp, int g, int L, bool vec_ok, float (&v)[16]) {
  const int col = grp * 4 + g;
  if (col >= cs) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = 0.0f;
    return;
  }
  const int gc = c0 + col;
  const float* p = gc < a.d ? reinterpret_cast<const float*>(a.A) + (int64_t)gc * a.lda
                            : reinterpret_cast<const float*>(a.b) + (int64_t)(gc - a.d) * a.ldb;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t j = tile + 4 * L + 64 * k;
    if (vec_ok && j + 3 < a.n) {
      const float4 x = *reinterpret_cast<const float4*>(p + j);
      v[4 * k + 0] = x.x;
      v[4 * k + 1] = x.y;
      v[4 * k + 2] = x.z;
      v[4 * k + 3] = x.w;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[4 * k + i] = (j + i < a.n) ? p[j + i] : 0.0f;
    }
  }
}

}  // namespace

__device__ __forceinline__ void acc_add(double* p, float v) { atomicAdd(p, (double)v); }

// Rows [4 i, 4 i + 4) of the table, local row 0 at global row row0g.  Rows 2m
// and 2m + 1 of one block hold stacked positions 2c and 2c + 1 of both
// halves, so one Philox call per half serves two rows.  Key word of a row:
// bucket of the H copy in bits 0-14, the sign bit of D(j) in bit 15, bucket
// of the I copy in bits 16-30 (r1 <= 32768).
__global__ void pi1_table_kernel(uint64_t seed, uint32_t instance, int64_t row0g, int64_t groups,
                                 int log2s, uint32_t r1, float scale_h, int sign_flip,
                                 uint4* __restrict__ keys, float4* __restrict__ cc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= groups) return;
  const uint64_t s = 1ull << log2s;
  const uint64_t j0 = (uint64_t)row0g + 4 * (uint64_t)i;
  const uint64_t kA = h_position(j0, log2s), kB = h_position(j0 + 2, log2s);
  const uint4 wa = stream_words(seed, kStreamPi1, kA >> 1, instance);
  const uint4 wb = stream_words(seed, kStreamPi1, kB >> 1, instance);
  const uint4 xa = stream_words(seed, kStreamPi1, (kA + s) >> 1, instance);
  const uint4 xb = stream_words(seed, kStreamPi1, (kB + s) >> 1, instance);
  // signs D(j0 .. j0 + 3): 4 bits of word (j0 / 32) % 4 of call j0 / 128
  uint32_t sg = 0;
  if (sign_flip) {
    const uint4 sw = stream_words(seed, kStreamSign, j0 >> 7, instance);
    const uint32_t sel = (uint32_t)(j0 >> 5) & 3u;
    const uint32_t word = sel == 0 ? sw.x : sel == 1 ? sw.y : sel == 2 ? sw.z : sw.w;
    sg = (word >> (j0 & 31u)) & 0xFu;
  }
  keys[i] = make_uint4(bucket_from_word(wa.x, r1) | ((sg & 1u) << 15) | (bucket_from_word(xa.x, r1) << 16),
                       bucket_from_word(wa.z, r1) | (((sg >> 1) & 1u) << 15) | (bucket_from_word(xa.z, r1) << 16),
                       bucket_from_word(wb.x, r1) | (((sg >> 2) & 1u) << 15) | (bucket_from_word(xb.x, r1) << 16),
                       bucket_from_word(wb.z, r1) | (((sg >> 3) & 1u) << 15) | (bucket_from_word(xb.z, r1) << 16));
  cc[2 * i] = make_float4(cauchy_from_word(wa.y) * scale_h, cauchy_from_word(xa.y) * 4.0f,
                          cauchy_from_word(wa.w) * scale_h, cauchy_from_word(xa.w) * 4.0f);
  cc[2 * i + 1] = make_float4(cauchy_from_word(wb.y) * scale_h, cauchy_from_word(xb.y) * 4.0f,
                              cauchy_from_word(wb.w) * scale_h, cauchy_from_word(xb.w) * 4.0f);
}

__global__ void __launch_bounds__(kWaves * 64) pass1_wave_kernel(Pass1Args a, int vec_ok) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c0 = blockIdx.y * a.c;
  const int cs = min(a.c, a.q - c0);
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int stride = pass1_acc_stride(cs);  // accumulator row stride (see its definition)
  const size_t acc_bytes =
      (((size_t)a.r1 * pass1_acc_stride(a.c) * sizeof(double)) + 15) & ~size_t(15);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveLds& W = reinterpret_cast<WaveLds*>(smem_raw + acc_bytes)[wave];
  for (int i = threadIdx.x; i < a.r1 * stride; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();

  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_range;
  const int64_t row1 = min(a.n_pad, row0 + a.rows_per_range);
  const int64_t sub = a.rows_per_range / kWaves;
  const int64_t w0 = row0 + wave * sub;
  const int64_t w1 = min(row1, w0 + sub);
  const int g = lane >> 4, L = lane & 15;
  const int ngroups = (cs + 3) >> 2;
  const bool vok = vec_ok != 0;

  float v[16], vn[16];
  uint4 tk = make_uint4(0, 0, 0, 0);
  float4 tc0 = make_float4(0.f, 0.f, 0.f, 0.f), tc1 = tc0;
  if (w0 < w1) {
    load_group(a, c0, cs, w0, 0, g, L, vok, v);
    const int64_t t4 = (w0 >> 2) + lane;
    tk = a.tab_keys[t4];
    tc0 = a.tab_c[2 * t4];
    tc1 = a.tab_c[2 * t4 + 1];
  }
  int64_t sign_base = w0;

  for (int64_t tile = w0; tile < w1; tile += kTile) {
    if (a.sign_flip && ((tile - w0) % kSignRows) == 0) {
      sign_base = tile;
      if (lane < kSignRows / 128) {
        const uint4 sw = stream_words(a.seed, kStreamSign, (uint64_t)((a.row0g + tile) >> 7) + lane,
                                      a.instance);
        *reinterpret_cast<uint4*>(&W.sgn[4 * lane]) = sw;
      }
    }
    {
      // table entries of rows tile + 4 lane + {0, 1, 2, 3}; then the next tile's
      const uint32_t ucs = (uint32_t)stride;  // the LDS table holds bucket * stride, the row offset
      uint4* eh = reinterpret_cast<uint4*>(&W.entH[4 * lane]);
      uint4* ei = reinterpret_cast<uint4*>(&W.entI[4 * lane]);
      eh[0] = make_uint4(__umul24(tk.x & 0x7FFFu, ucs), __float_as_uint(tc0.x),
                         __umul24(tk.y & 0x7FFFu, ucs), __float_as_uint(tc0.z));
      eh[1] = make_uint4(__umul24(tk.z & 0x7FFFu, ucs), __float_as_uint(tc1.x),
                         __umul24(tk.w & 0x7FFFu, ucs), __float_as_uint(tc1.z));
      ei[0] = make_uint4(__umul24(tk.x >> 16, ucs), __float_as_uint(tc0.y),
                         __umul24(tk.y >> 16, ucs), __float_as_uint(tc0.w));
      ei[1] = make_uint4(__umul24(tk.z >> 16, ucs), __float_as_uint(tc1.y),
                         __umul24(tk.w >> 16, ucs), __float_as_uint(tc1.w));
      if (tile + kTile < w1) {
        const int64_t t4 = ((tile + kTile) >> 2) + lane;
        tk = a.tab_keys[t4];
        tc0 = a.tab_c[2 * t4];
        tc1 = a.tab_c[2 * t4 + 1];
      }
    }
    wave_sync();
    const int soff = (int)((tile - sign_base) >> 5);

    for (int grp = 0; grp < ngroups; ++grp) {
      if (grp + 1 < ngroups) load_group(a, c0, cs, tile, grp + 1, g, L, vok, vn);
      else if (tile + kTile < w1) load_group(a, c0, cs, tile + kTile, 0, g, L, vok, vn);
      const int colr = grp * 4 + g;
      const bool cact = colr < cs;
      const int col = cact ? colr : cs - 1;  // idle lanes (masked off at the adds) stay in bounds
      // sign D(j) (and the minus of the b column) as a sign-bit xor
      const uint32_t negb = (cact && a.b && c0 + col >= a.d) ? 0x80000000u : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        uint32_t bits = 0;
        if (a.sign_flip) bits = (W.sgn[soff + (L >> 3) + 2 * k] >> ((L & 7) * 4)) & 0xFu;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t m = (((bits >> i) & 1u) << 31) ^ negb;
          v[4 * k + i] = __uint_as_float(__float_as_uint(v[4 * k + i]) ^ m);
        }
      }
      // I-half copies: rows t = 4 L + i + 64 k
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t0 = 4 * L + 64 * k;
        const uint4 e01 = *reinterpret_cast<const uint4*>(&W.entI[t0]);
        const uint4 e23 = *reinterpret_cast<const uint4*>(&W.entI[t0 + 2]);
        if (cact) {
          acc_add(&acc[e01.x + col], __uint_as_float(e01.y) * v[4 * k + 0]);
          acc_add(&acc[e01.z + col], __uint_as_float(e01.w) * v[4 * k + 1]);
          acc_add(&acc[e23.x + col], __uint_as_float(e23.y) * v[4 * k + 2]);
          acc_add(&acc[e23.z + col], __uint_as_float(e23.w) * v[4 * k + 3]);
        }
      }
      // butterflies over row bits 0, 1 (register bits 0, 1) and 6, 7 (register bits 2, 3)
      if (a.log2s > 0) reg_stage(v, 0);
      if (a.log2s > 1) reg_stage(v, 1);
      if (a.log2s > 6) reg_stage(v, 2);
      if (a.log2s > 7) reg_stage(v, 3);
      // butterflies over row bits 2-5, held in the lane index, across lanes
      if (a.log2s > 2) lane_stage<0>(v, L);
      if (a.log2s > 3) lane_stage<1>(v, L);
      if (a.log2s > 4) lane_stage<2>(v, L);
      if (a.log2s > 5) lane_stage<3>(v, L);
      // H-half copies: rows t = 4 L + i + 64 k, as for the I half
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t0 = 4 * L + 64 * k;
        const uint4 e01 = *reinterpret_cast<const uint4*>(&W.entH[t0]);
        const uint4 e23 = *reinterpret_cast<const uint4*>(&W.entH[t0 + 2]);
        if (cact) {
          acc_add(&acc[e01.x + col], __uint_as_float(e01.y) * v[4 * k + 0]);
          acc_add(&acc[e01.z + col], __uint_as_float(e01.w) * v[4 * k + 1]);
          acc_add(&acc[e23.x + col], __uint_as_float(e23.y) * v[4 * k + 2]);
          acc_add(&acc[e23.z + col], __uint_as_float(e23.w) * v[4 * k + 3]);
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = vn[r];
    }
    wave_sync();  // table and sign words are rewritten by the next tile
  }
  __syncthreads();
  float* part = reinterpret_cast<float*>(a.partials);
  for (int col = 0; col < cs; ++col) {
    float* dst = part + ((size_t)blockIdx.x * a.q + c0 + col) * a.r1;
    for (int i = threadIdx.x; i < a.r1; i += blockDim.x) dst[i] = (float)acc[i * stride + col];
  }
}

__global__ void __launch_bounds__(kWaves * 64) pass1_block_kernel(Pass1Args a, int vec_ok) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int c0 = blockIdx.y * a.c;
  const int cs = min(a.c, a.q - c0);
  double* acc = reinterpret_cast<double*>(smem_raw);
  const int stride = pass1_acc_stride(cs);  // accumulator row stride (see its definition)
  const size_t acc_bytes =
      (((size_t)a.r1 * pass1_acc_stride(a.c) * sizeof(double)) + 15) & ~size_t(15);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveTab& W = reinterpret_cast<WaveTab*>(smem_raw + acc_bytes)[wave];
  float* xch = reinterpret_cast<float*>(smem_raw + acc_bytes + kWaves * sizeof(WaveTab));
  for (int i = threadIdx.x; i < a.r1 * stride; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();

  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_range;
  const int64_t row1 = min(a.n_pad, row0 + a.rows_per_range);
  const int g = lane >> 4, L = lane & 15;
  const int ngroups = (cs + 3) >> 2;
  const bool vok = vec_ok != 0;
  constexpr int64_t kStep = (int64_t)kWaves * kTile;

  // The workgroup walks its range in steps of kWaves tiles, wave w taking
  // tile w of each step, so that a block of s rows spans the s / kTile
  // neighbouring waves whose Hadamard stages over row bits >= 8 meet in LDS.
  // Every wave takes the same number of steps (the barriers rely on it).
  const int64_t niter = (a.rows_per_range + kStep - 1) / kStep;
  const int64_t tbase = row0 + (int64_t)kTile * wave;
  const int64_t tstride = kStep;
  float v[16], vn[16];
  uint4 tk = make_uint4(0, 0, 0, 0);
  float4 tc0 = make_float4(0.f, 0.f, 0.f, 0.f), tc1 = tc0;
  {
    const int64_t t0 = tbase;
    if (t0 < row1) {
      load_group(a, c0, cs, t0, 0, g, L, vok, v);
      const int64_t t4 = (t0 >> 2) + lane;
      tk = a.tab_keys[t4];
      tc0 = a.tab_c[2 * t4];
      tc1 = a.tab_c[2 * t4 + 1];
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = 0.0f;
    }
  }

  for (int64_t it = 0; it < niter; ++it) {
    const int64_t tile = tbase + it * tstride;
    const int64_t next = tile + tstride;
    const bool act = tile < row1;                      // whole blocks of s rows share this
    const bool more = it + 1 < niter && next < row1;  // this wave's next tile exists
    if (act) {
      // table entries of rows tile + 4 lane + {0, 1, 2, 3}; then the next tile's
      const uint32_t ucs = (uint32_t)stride;  // the LDS table holds bucket * stride, the row offset
      uint4* eh = reinterpret_cast<uint4*>(&W.entH[4 * lane]);
      uint4* ei = reinterpret_cast<uint4*>(&W.entI[4 * lane]);
      // I entries carry the sign of D(j) (bit 15 of the key) in bit 31
      eh[0] = make_uint4(__umul24(tk.x & 0x7FFFu, ucs), __float_as_uint(tc0.x),
                         __umul24(tk.y & 0x7FFFu, ucs), __float_as_uint(tc0.z));
      eh[1] = make_uint4(__umul24(tk.z & 0x7FFFu, ucs), __float_as_uint(tc1.x),
                         __umul24(tk.w & 0x7FFFu, ucs), __float_as_uint(tc1.z));
      ei[0] = make_uint4(__umul24(tk.x >> 16, ucs) | ((tk.x & 0x8000u) << 16), __float_as_uint(tc0.y),
                         __umul24(tk.y >> 16, ucs) | ((tk.y & 0x8000u) << 16), __float_as_uint(tc0.w));
      ei[1] = make_uint4(__umul24(tk.z >> 16, ucs) | ((tk.z & 0x8000u) << 16), __float_as_uint(tc1.y),
                         __umul24(tk.w >> 16, ucs) | ((tk.w & 0x8000u) << 16), __float_as_uint(tc1.w));
      if (more) {
        const int64_t t4 = (next >> 2) + lane;
        tk = a.tab_keys[t4];
        tc0 = a.tab_c[2 * t4];
        tc1 = a.tab_c[2 * t4 + 1];
      }
    }
    wave_sync();

    for (int grp = 0; grp < ngroups; ++grp) {
      if (grp + 1 < ngroups) {
        if (act) load_group(a, c0, cs, tile, grp + 1, g, L, vok, vn);
      } else if (more) {
        load_group(a, c0, cs, next, 0, g, L, vok, vn);
      }
      const int colr = grp * 4 + g;
      const bool cact = act && colr < cs;  // lanes with nothing to add are masked off
      const int col = cact ? colr : cs - 1;  // idle lanes (masked off at the adds) stay in bounds
      // sign D(j) (bit 31 of the I entry) and the minus of the b column as a
      // sign-bit xor, then the I-half copies: rows t = 4 L + i + 64 k
      const uint32_t negb = (cact && a.b && c0 + col >= a.d) ? 0x80000000u : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t0 = 4 * L + 64 * k;
        const uint4 e01 = *reinterpret_cast<const uint4*>(&W.entI[t0]);
        const uint4 e23 = *reinterpret_cast<const uint4*>(&W.entI[t0 + 2]);
        const uint32_t off[4] = {e01.x, e01.z, e23.x, e23.z};
        const uint32_t cw[4] = {e01.y, e01.w, e23.y, e23.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t m = (off[i] & 0x80000000u) ^ negb;
          v[4 * k + i] = __uint_as_float(__float_as_uint(v[4 * k + i]) ^ m);
          if (cact) acc_add(&acc[(off[i] & 0x7FFFFFFFu) + col], __uint_as_float(cw[i]) * v[4 * k + i]);
        }
      }
      // butterflies over row bits 0, 1 (register bits 0, 1) and 6, 7 (register bits 2, 3)
      if (a.log2s > 0) reg_stage(v, 0);
      if (a.log2s > 1) reg_stage(v, 1);
      if (a.log2s > 6) reg_stage(v, 2);
      if (a.log2s > 7) reg_stage(v, 3);
      // butterflies over row bits 2-5, held in the lane index, across lanes
      if (a.log2s > 2) lane_stage<0>(v, L);
      if (a.log2s > 3) lane_stage<1>(v, L);
      if (a.log2s > 4) lane_stage<2>(v, L);
      if (a.log2s > 5) lane_stage<3>(v, L);
      // row bits >= 8 live in the wave index: each stage pairs wave w with
      // w ^ (1 << (bit - 8)) through the exchange buffers (the lower-row wave
      // keeps a + b, the upper one b - a)
      for (int bit = 8; bit < a.log2s; ++bit) {
        const int pw = wave ^ (1 << (bit - 8));
        const bool upper = (wave >> (bit - 8)) & 1;
        float* mine = xch + wave * kXch;
        const float* theirs = xch + pw * kXch;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int r = 0; r < 8; ++r) mine[r * 64 + lane] = v[8 * h + r];
          __syncthreads();
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const float o = theirs[r * 64 + lane];
            v[8 * h + r] = upper ? o - v[8 * h + r] : v[8 * h + r] + o;
          }
          __syncthreads();
        }
      }
      // H-half copies: rows t = 4 L + i + 64 k, as for the I half
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t0 = 4 * L + 64 * k;
        const uint4 e01 = *reinterpret_cast<const uint4*>(&W.entH[t0]);
        const uint4 e23 = *reinterpret_cast<const uint4*>(&W.entH[t0 + 2]);
        if (cact) {
          acc_add(&acc[e01.x + col], __uint_as_float(e01.y) * v[4 * k + 0]);
          acc_add(&acc[e01.z + col], __uint_as_float(e01.w) * v[4 * k + 1]);
          acc_add(&acc[e23.x + col], __uint_as_float(e23.y) * v[4 * k + 2]);
          acc_add(&acc[e23.z + col], __uint_as_float(e23.w) * v[4 * k + 3]);
        }
      }
      const bool have_next = grp + 1 < ngroups ? act : more;
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = have_next ? vn[r] : 0.0f;
    }
    wave_sync();  // table and sign words are rewritten by the next tile
  }
  __syncthreads();
  float* part = reinterpret_cast<float*>(a.partials);
  for (int col = 0; col < cs; ++col) {
    float* dst = part + ((size_t)blockIdx.x * a.q + c0 + col) * a.r1;
    for (int i = threadIdx.x; i < a.r1; i += blockDim.x) dst[i] = (float)acc[i * stride + col];
  }
}

size_t pass1_wave_lds(int r1, int stride, int s) {
  const size_t acc = (((size_t)r1 * stride * sizeof(double)) + 15) & ~size_t(15);
  if (s > kTile) return acc + kWaves * (sizeof(WaveTab) + (size_t)kXch * sizeof(float));
  return acc + kWaves * sizeof(WaveLds);
}

int pass1_wave_rows_quantum() { return kWaves * kTile; }

int64_t pi1_table_rows(int64_t n_pad) { return (n_pad + kTile - 1) / kTile * kTile; }

hipError_t launch_pi1_table(uint64_t seed, uint32_t instance, int64_t row0g, int64_t rows, int s,
                            int r1, int sign_flip, uint4* keys, float4* cc, hipStream_t st) {
  const int64_t groups = rows / 4;
  const unsigned blocks = (unsigned)((groups + 255) / 256);
  int log2s = 0;
  while ((1 << log2s) < s) ++log2s;
  hipLaunchKernelGGL(pi1_table_kernel, dim3(blocks), dim3(256), 0, st, seed, instance, row0g,
                     groups, log2s, (uint32_t)r1, 4.0f / sqrtf((float)s), sign_flip, keys, cc);
  return hipGetLastError();
}

bool pass1_wave_signs_in_table(int s) { return s > kTile; }

hipError_t launch_pass1_wave(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st) {
  const void* fn = a.s > kTile ? (const void*)pass1_block_kernel : (const void*)pass1_wave_kernel;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
  if (e != hipSuccess) return e;
  if (a.s > kTile)
    hipLaunchKernelGGL(pass1_block_kernel, dim3(p.nranges, p.nslices), dim3(kWaves * 64), p.lds,
                       st, a, vec_ok ? 1 : 0);
  else
    hipLaunchKernelGGL(pass1_wave_kernel, dim3(p.nranges, p.nslices), dim3(kWaves * 64), p.lds, st,
                       a, vec_ok ? 1 : 0);
  return hipGetLastError();
}

}  // namespace fctl1
