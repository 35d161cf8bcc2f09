// Pass 1, bucket-owner form, for FP32 data and s <= 1024: Y = Pi1 X with
// Pi1 = 4 B C H~ (section "FCT1 Construction": n/s Hadamard transforms of size
// s, a diagonal Cauchy scaling C and a hash B with one non-zero per stacked
// position).
//
// A workgroup of 8 waves owns a range of whole 8192-row tiles, a slice of at
// most 18 (24) columns of X = [A, -b] and a range of at most 1024 (512) buckets
// (rows of Y).  Lane t owns one or two of those buckets.  Per tile:
//   1. each wave draws the random part of Pi1 for its 1024 rows: D(j) for
//      every row, and bucket and Cauchy of both stacked copies of every row,
//      one Philox call per pair of positions.  The I-half copy of a row is
//      kept by the lane that loads the row, the H-half copy by the lane that
//      holds that entry of H u after the butterflies (fwht_span1024);
//   2. the tile's 16384 positions are counted per wave and bucket into LDS;
//      the ranks come back from the counter adds, so they follow the wave's
//      own instruction and lane order.  A workgroup scan turns the counts into
//      offsets of a staging array sorted by bucket (bucket-major, wave-minor),
//      every bucket's segment padded to an even length with a zero, and every
//      position keeps its slot;
//   3. for each column of the slice every wave loads its rows (float4), applies
//      D (and the minus sign of the b column), stores 4 C_k u of each I-half
//      copy into its slot, runs the butterflies, and stores
//      4 C_k (H u) / sqrt(s) of each H-half copy into its slot; after a barrier
//      lane t sums its buckets' segments in slot order (FP32 when a bucket
//      takes at most about 64 positions of a tile, FP64 otherwise) and adds
//      the sums into its FP32 accumulators for that column (registers).
//      Columns alternate between two staging arrays, so one barrier per
//      column separates writers and readers, and half of the waves sum a
//      column before producing the next one while the other half produce
//      first, which overlaps sums and butterflies on every SIMD.
// Nothing is added atomically to a sum: every sum is formed by one lane in an
// order fixed by the random streams, so the sketch is the same bit for bit on
// every run.  The accumulators are written once per workgroup as FP32
// partials, which the reduction kernel adds in a fixed order.  Rows past the
// padded end of X are loaded as zeros and add exact zeros.
#include <type_traits>

#include "fct_device.h"
#include "fct_kernels.h"
#include "wave_fwht.h"

namespace fctl1 {

namespace {

constexpr int kOW = 8;                   // waves per workgroup
constexpr int kOT = kOW * 64;            // threads per workgroup
constexpr int kORowsWave = 1024;         // rows per wave per tile
constexpr int kOTile = kOW * kORowsWave; // rows per tile
constexpr int kOPos = 2 * kOTile;        // stacked positions per tile
constexpr int kOColsNB2 = 18;            // columns per slice when a lane owns two buckets
constexpr int kOColsNB1 = 24;            // ... one bucket

struct OwnLayout {
  uint32_t stage, stage_bytes, cnt, sgn, wsum, total;
};

__host__ __device__ inline uint32_t al16(uint32_t v) { return (v + 15u) & ~15u; }

// LDS carve for `span` buckets: two bucket-sorted staging arrays (columns
// alternate between them; every segment padded to even length, plus a
// discard slot), per-wave counters (two 16-bit counters
// per word when a lane owns two buckets, plus a spare word for positions
// outside the workgroup's bucket range), per-wave sign words and the scan's
// wave totals.
__host__ __device__ inline OwnLayout own_layout(int span) {
  const int nb = span > 512 ? 2 : 1;
  const int cw = nb == 2 ? (span + 1) / 2 : span;
  OwnLayout L;
  uint32_t o = 0;
  L.stage = o;
  L.stage_bytes = al16((uint32_t)(kOPos + span + 4) * 4u);
  o += 2 * L.stage_bytes;
  L.cnt = o;
  o += al16((uint32_t)(kOW * (cw + 1)) * 4u);
  L.sgn = o;
  o += kOW * 32 * 4;
  L.wsum = o;
  o += 64;
  L.total = o;
  return L;
}

__device__ __forceinline__ void own_load(const Pass1Args& a, int gc, int64_t tl, int lane, bool vok,
                                         float (&v)[16]) {
  const float* p = gc < a.d ? reinterpret_cast<const float*>(a.A) + (int64_t)gc * a.lda
                            : reinterpret_cast<const float*>(a.b) + (int64_t)(gc - a.d) * a.ldb;
  if (vok && tl + kORowsWave <= a.n) {  // the wave's whole span is inside X (wave-uniform)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 x = *reinterpret_cast<const float4*>(p + tl + 4 * lane + 256 * k);
      v[4 * k + 0] = x.x;
      v[4 * k + 1] = x.y;
      v[4 * k + 2] = x.z;
      v[4 * k + 3] = x.w;
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t j = tl + 4 * lane + 256 * k;
    if (vok && j + 3 < a.n) {
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

// Exclusive scan over the workgroup of one value per thread (wave scans by
// shuffles, then the wave totals through LDS).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* wsum, int wave, int lane) {
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int w = 0; w < kOW; ++w)
    if (w < wave) before += wsum[w];
  return before + incl - x;
}

// bucket (local to the workgroup's bucket range, in bits 16-31; all ones when
// outside it) and pre-scaled Cauchy of one stacked position
__device__ __forceinline__ void own_position(uint32_t wb, uint32_t wc, uint32_t r1, int blo, int span,
                                             float scale, uint32_t& key, float& cv) {
  const int lb = (int)bucket_from_word(wb, r1) - blo;
  key = (lb >= 0 && lb < span) ? ((uint32_t)lb << 16) : 0xFFFFFFFFu;
  cv = cauchy_from_word(wc) * scale;
}

}  // namespace

// Producer half of a column: take the column's loaded values v (consumed),
// apply D and the sign of the b column, store 4 C_k u of the I-half copies
// into their slots of staging array `sb`, run the butterflies, store
// 4 C_k (H u) / sqrt(s) of the H-half copies.
template <int LOG2S>
__device__ __forceinline__ void own_produce(const Pass1Args& a, unsigned char* sb, int col, int c0,
                                           int L, const uint32_t (&sm)[16], const float (&cI)[16],
                                           const float (&cH)[16], const uint32_t (&slI)[16],
                                           const uint32_t (&slH)[16], float (&v)[16]) {
  const uint32_t negb = (a.b && c0 + col >= a.d) ? 0x80000000u : 0u;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    v[r] = __uint_as_float(xor3(__float_as_uint(v[r]), sm[r], negb));
    *reinterpret_cast<float*>(sb + slI[r]) = cI[r] * v[r];
  }
  fwht_span1024_dpp<LOG2S>(v, L);
#pragma unroll
  for (int r = 0; r < 16; ++r) *reinterpret_cast<float*>(sb + slH[r]) = cH[r] * v[r];
}

// Accumulators of one bucket for the columns of a slice, held in registers
// and indexed by the (wave-uniform) column: a vector of 16 for columns 0-15
// and one of HI for the rest.  A uniform index into such a vector is a
// relative register move (s_set_gpr_idx), not a scratch access.  They are
// FP32: a workgroup adds the sums of at most 64 tiles (16 unless the rows
// would need more than 4096 ranges), so with segments of at most about 64
// terms summed in two chains a bucket's sum is within about 100 u of its l1
// mass; the ranges' partials are added in FP64.
typedef float fvec16 __attribute__((ext_vector_type(16)));
typedef float fvec8 __attribute__((ext_vector_type(8)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

template <int CMAX> struct ColAcc {
  static_assert(CMAX == 18 || CMAX == 24, "slice widths of the owner kernel");
  using Hi = typename std::conditional<CMAX == 18, fvec2, fvec8>::type;
  fvec16 lo;
  Hi hi;
  __device__ __forceinline__ void zero() {
    lo = 0.0f;
    hi = 0.0f;
  }
  __device__ __forceinline__ void add(int col, float x) {
    if (col < 16) lo[col] += x;
    else hi[col - 16] += x;
  }
  __device__ __forceinline__ float get(int col) const { return col < 16 ? lo[col] : hi[col - 16]; }
};

// Owner half of a column: the sums of this lane's buckets' segments of
// staging array `sb`, in slot order, added into the column's accumulators.
template <int NB, int CMAX>
__device__ __forceinline__ void own_sum(const unsigned char* sb, int col, int span,
                                       const uint32_t (&seg0)[NB], const uint32_t (&seg1)[NB],
                                       ColAcc<CMAX> (&m)[NB]) {
  const float2* st2 = reinterpret_cast<const float2*>(sb);
  float sacc[NB];
  if (span >= 256) {
    // about 2 * 8192 / span <= 64 terms per segment: FP32 (two chains, even
    // and odd slots) is within 64 u of the segment's l1 mass
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      float se = 0.0f, so = 0.0f;
#pragma unroll 4
      for (uint32_t q2 = seg0[u] >> 1; q2 < (seg1[u] >> 1); ++q2) {
        const float2 x = st2[q2];
        se += x.x;
        so += x.y;
      }
      sacc[u] = se + so;
    }
  } else {
    // long segments (few buckets): FP64
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      double se = 0.0, so = 0.0;
#pragma unroll 4
      for (uint32_t q2 = seg0[u] >> 1; q2 < (seg1[u] >> 1); ++q2) {
        const float2 x = st2[q2];
        se += (double)x.x;
        so += (double)x.y;
      }
      sacc[u] = (float)(se + so);
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) m[u].add(col, sacc[u]);
}

template <int NB, int LOG2S>
__global__ void __launch_bounds__(kOT) pass1_owner_kernel(Pass1Args a, int vec_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int CMAX = NB == 2 ? kOColsNB2 : kOColsNB1;
  constexpr uint32_t S = 1u << LOG2S;
  const int c0 = blockIdx.y * a.c;
  const int cs = min(a.c, a.q - c0);
  const int blo = blockIdx.z * a.bucket_span;
  const int span = min(a.bucket_span, a.r1 - blo);
  const int cw = NB == 2 ? (span + 1) >> 1 : span;  // counter words per wave (+1 spare below)
  const OwnLayout Ly = own_layout(a.bucket_span);
  float* stage = reinterpret_cast<float*>(smem + Ly.stage);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem + Ly.cnt);
  uint32_t* sgn = reinterpret_cast<uint32_t*>(smem + Ly.sgn);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + Ly.wsum);
  // a position whose bucket is outside the workgroup's range is counted in a
  // spare counter word and stored into a discard slot
  const uint32_t trash = 4u * (uint32_t)(kOPos + span);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, L = lane & 15;
  const bool vok = vec_ok != 0;
  // 4 / sqrt(s) and the sign the butterflies leave in this lane
  const float scale_h = a.scale_h * span_sign(L, LOG2S);
  uint32_t* mycnt = cnt + wave * (cw + 1);

  ColAcc<CMAX> m[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) m[u].zero();

  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_range;
  const int64_t tiles_end = (a.n_pad + kOTile - 1) / kOTile * kOTile;
  const int64_t row1 = min(tiles_end, row0 + a.rows_per_range);

  float v[16], cI[16], cH[16];
  uint32_t sm[16], slI[16], slH[16];

  for (int64_t tile = row0; tile < row1; tile += kOTile) {
    const int64_t tl = tile + (int64_t)wave * kORowsWave;  // window-local first row of this wave
    const uint64_t jg0 = (uint64_t)a.row0g + (uint64_t)tl;  // its global row (a multiple of s)
    own_load(a, c0, tl, lane, vok, v);                      // column 0, in flight during set-up

    // ---- set-up of the tile (independent of X) ----
    for (int i = tid; i < kOW * (cw + 1); i += kOT) cnt[i] = 0u;
    if (a.sign_flip && lane < 8) {
      const uint4 sw = stream_words(a.seed, kStreamSign, (jg0 >> 7) + (uint64_t)lane, a.instance);
      *reinterpret_cast<uint4*>(&sgn[wave * 32 + 4 * lane]) = sw;
    }
    // Bucket and Cauchy of the 32 positions, one pair of rows per step: the
    // I-half copies, then the H-half ones, each half through this thread's
    // 16 slots of the staging area (unused until the columns start), so that
    // only one step's values are live at a time.  Row jg0 + t of the wave's
    // span has its H-half copy at 2 jg0 + 2 s (t >> log2 s) + (t mod s): jg0
    // is a multiple of s, so the call index is jg0 plus a 32-bit offset.
    {
      uint2* scr = reinterpret_cast<uint2*>(stage);
      int lane_o = lane;
      asm volatile("" : "+v"(lane_o));  // keeps the per-lane row offsets inside the tile loop
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
#pragma unroll 1
        for (int g = 0; g < 8; ++g) {
          const int k = g >> 1, p = g & 1, r = 4 * k + 2 * p;
          const uint32_t t = hh ? (uint32_t)span_row_out_dpp(lane_o, r, LOG2S)
                                : (uint32_t)(2 * p + 4 * lane_o + 256 * k);
          const uint32_t hloc = ((t >> LOG2S) << (LOG2S + 1)) + (t & (S - 1)) + (hh ? 0u : S);
          const uint4 w = stream_words(a.seed, kStreamPi1, jg0 + (hloc >> 1), a.instance);
          const float sc = hh ? scale_h : 4.0f;
          uint32_t k0, k1;
          float c0v, c1v;
          own_position(w.x, w.y, (uint32_t)a.r1, blo, span, sc, k0, c0v);
          own_position(w.z, w.w, (uint32_t)a.r1, blo, span, sc, k1, c1v);
          scr[(2 * g) * kOT + tid] = make_uint2(k0, __float_as_uint(c0v));
          scr[(2 * g + 1) * kOT + tid] = make_uint2(k1, __float_as_uint(c1v));
        }
        // register r = 4 k + 2 p + e was step g = 2 k + p, slot 2 g + e
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int g = 2 * (r >> 2) + ((r >> 1) & 1);
          const uint2 x = scr[(2 * g + (r & 1)) * kOT + tid];
          if (hh) {
            slH[r] = x.x;
            cH[r] = __uint_as_float(x.y);
          } else {
            slI[r] = x.x;
            cI[r] = __uint_as_float(x.y);
          }
        }
      }
    }
    wave_sync();
    if (a.sign_flip) {
      // row t = i + 4 lane + 256 k: word (t >> 5) = (lane >> 3) + 8 k, bit 4 (lane & 7) + i
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t word = sgn[wave * 32 + (lane >> 3) + 8 * k];
#pragma unroll
        for (int i = 0; i < 4; ++i) sm[4 * k + i] = ((word >> (4 * (lane & 7) + i)) & 1u) << 31;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) sm[r] = 0u;
    }
    __syncthreads();  // counters cleared

    // ranks within (wave, bucket), from the counter adds; keys outside the
    // bucket range count in the spare word cw
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint32_t& key = h ? slH[r] : slI[r];
        const uint32_t lb = key >> 16;  // 0xFFFF outside the range
        const uint32_t word = NB == 2 ? min(lb >> 1, (uint32_t)cw) : min(lb, (uint32_t)cw);
        const uint32_t sh = NB == 2 ? (lb & 1u) << 4 : 0u;
        const uint32_t old = atomicAdd(&mycnt[word], 1u << sh);
        key = (key & 0xFFFF0000u) | (NB == 2 ? __builtin_amdgcn_ubfe(old, sh, 16) : (old & 0xFFFFu));
      }
    __syncthreads();  // counts complete

    // bucket-major, wave-minor offsets; lane t owns buckets NB t .. NB t + NB - 1
    uint32_t seg0[NB], seg1[NB];
    {
      uint32_t tot[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) tot[u] = 0u;
      if (tid < cw) {
#pragma unroll
        for (int w = 0; w < kOW; ++w) {
          const uint32_t cv = cnt[w * (cw + 1) + tid];
          if (NB == 2) {
            tot[0] += cv & 0xFFFFu;
            tot[NB - 1] += cv >> 16;
          } else {
            tot[0] += cv;
          }
        }
      }
      uint32_t padded[NB], sum = 0u;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        padded[u] = (tot[u] + 1u) & ~1u;
        sum += padded[u];
      }
      uint32_t base = block_excl_scan(sum, wsum, wave, lane);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        seg0[u] = base;
        seg1[u] = base + padded[u];
        if (tot[u] & 1u) {  // pad the segment with a zero, in both staging arrays
          stage[base + tot[u]] = 0.0f;
          stage[Ly.stage_bytes / 4 + base + tot[u]] = 0.0f;
        }
        base += padded[u];
      }
      if (tid < cw) {
        uint32_t run[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) run[u] = seg0[u];
#pragma unroll
        for (int w = 0; w < kOW; ++w) {
          const uint32_t cv = cnt[w * (cw + 1) + tid];
          if (NB == 2) {
            cnt[w * (cw + 1) + tid] = run[0] | (run[NB - 1] << 16);
            run[0] += cv & 0xFFFFu;
            run[NB - 1] += cv >> 16;
          } else {
            cnt[w * (cw + 1) + tid] = run[0];
            run[0] += cv;
          }
        }
      }
    }
    __syncthreads();  // offsets complete
    // slots as byte offsets within a staging array
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint32_t& key = h ? slH[r] : slI[r];
        const uint32_t lb = key >> 16;
        const uint32_t word = NB == 2 ? min(lb >> 1, (uint32_t)cw) : min(lb, (uint32_t)cw);
        const uint32_t off = NB == 2 ? __builtin_amdgcn_ubfe(mycnt[word], (lb & 1u) << 4, 16)
                                     : mycnt[word];
        key = lb < (uint32_t)span ? 4u * (off + (key & 0xFFFFu)) : trash;
      }

    // ---- the slice's columns, alternating between the two staging arrays ----
    // Column col goes through array col & 1.  After the barrier that
    // completes column col, a wave sums column col and produces column
    // col + 1 into the other array, which is free: every wave finished its
    // sums of column col - 1 before that barrier.  Waves 0-3 sum first and
    // waves 4-7 produce first, so the two waves sharing a SIMD overlap the
    // LDS-bound sums with the VALU-bound butterflies.  The load of the next
    // column to produce goes into v as soon as v is consumed and is in flight
    // during a sum.
    own_produce<LOG2S>(a, smem + Ly.stage, 0, c0, L, sm, cI, cH, slI, slH, v);
    if (1 < cs) own_load(a, c0 + 1, tl, lane, vok, v);
    __syncthreads();
    const bool sum_first = wave < 4;
    for (int col = 0; col < cs; ++col) {
      unsigned char* cur = smem + Ly.stage + (col & 1) * Ly.stage_bytes;
      unsigned char* nxt = smem + Ly.stage + ((col + 1) & 1) * Ly.stage_bytes;
      if (sum_first) {
        own_sum<NB, CMAX>(cur, col, span, seg0, seg1, m);
        if (col + 1 < cs) {
          own_produce<LOG2S>(a, nxt, col + 1, c0, L, sm, cI, cH, slI, slH, v);
          if (col + 2 < cs) own_load(a, c0 + col + 2, tl, lane, vok, v);
        }
      } else {
        if (col + 1 < cs) {
          own_produce<LOG2S>(a, nxt, col + 1, c0, L, sm, cI, cH, slI, slH, v);
          if (col + 2 < cs) own_load(a, c0 + col + 2, tl, lane, vok, v);
        }
        own_sum<NB, CMAX>(cur, col, span, seg0, seg1, m);
      }
      __syncthreads();  // column col + 1 complete; column col's array free again
    }
  }

  float* part = reinterpret_cast<float*>(a.partials);
#pragma unroll
  for (int cc = 0; cc < CMAX; ++cc)
    if (cc < cs) {
      float* dst = part + ((size_t)blockIdx.x * a.q + c0 + cc) * a.r1 + blo;
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int bkt = NB * tid + u;
        if (bkt < span) dst[bkt] = m[u].get(cc);
      }
    }
}

int pass1_owner_max_cols(int span) { return span > 512 ? kOColsNB2 : kOColsNB1; }

size_t pass1_owner_lds(int span, int c) {
  (void)c;
  return own_layout(span).total;
}

int pass1_owner_tile_rows() { return kOTile; }

template <int NB>
static hipError_t launch_owner_nb(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st) {
  const void* fns[10] = {
      (const void*)pass1_owner_kernel<NB, 1>, (const void*)pass1_owner_kernel<NB, 2>,
      (const void*)pass1_owner_kernel<NB, 3>, (const void*)pass1_owner_kernel<NB, 4>,
      (const void*)pass1_owner_kernel<NB, 5>, (const void*)pass1_owner_kernel<NB, 6>,
      (const void*)pass1_owner_kernel<NB, 7>, (const void*)pass1_owner_kernel<NB, 8>,
      (const void*)pass1_owner_kernel<NB, 9>, (const void*)pass1_owner_kernel<NB, 10>};
  if (a.log2s < 1 || a.log2s > 10) return hipErrorInvalidValue;
  const void* fn = fns[a.log2s - 1];
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
  if (e != hipSuccess) return e;
  Pass1Args aa = a;
  int vo = vec_ok ? 1 : 0;
  void* args[] = {&aa, &vo};
  return hipLaunchKernel(fn, dim3(p.nranges, p.nslices, p.nbranges), dim3(kOT), args, p.lds, st);
}

hipError_t launch_pass1_owner(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st) {
  return a.bucket_span > 512 ? launch_owner_nb<2>(a, p, vec_ok, st)
                             : launch_owner_nb<1>(a, p, vec_ok, st);
}

}  // namespace fctl1
