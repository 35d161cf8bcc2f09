// Pass 1, bucket-owner form, for FP32 data and s <= 1024: Y = Pi1 X with
// Pi1 = 4 B C H~ (section "FCT1 Construction": n/s Hadamard transforms of size
// s, a diagonal Cauchy scaling C and a hash B with one non-zero per stacked
// position).
//
// A workgroup of 8 waves owns a range of whole 8192-row tiles, a slice of at
// most kOwnColsMax columns of X = [A, -b] and a range of at most 1024 buckets
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
//      takes at most about 64 positions of a tile, FP64 otherwise) and parks
//      the sums in LDS;
//   4. at the end of the tile lane t adds the parked sums into FP64 registers.
// Nothing is added atomically to a sum: every sum is formed by one lane in an
// order fixed by the random streams, so the sketch is the same bit for bit on
// every run.  The FP64 accumulators are written once per workgroup as FP32
// partials, which the reduction kernel adds in a fixed order.  Rows past the
// padded end of X are loaded as zeros and add exact zeros.
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
constexpr int kOColsNB1 = 32;            // ... one bucket

struct OwnLayout {
  uint32_t stage, cnt, tsum, sgn, wsum, total;
};

__host__ __device__ inline uint32_t al16(uint32_t v) { return (v + 15u) & ~15u; }

// LDS carve for `span` buckets and `c` columns: the bucket-sorted staging
// array (every segment padded to even length, plus a discard slot), per-wave
// counters (two 16-bit counters per word when a lane owns two buckets), the
// parked per-column sums, per-wave sign words and the scan's wave totals.
__host__ __device__ inline OwnLayout own_layout(int span, int c) {
  const int nb = span > 512 ? 2 : 1;
  const int cw = nb == 2 ? (span + 1) / 2 : span;
  OwnLayout L;
  uint32_t o = 0;
  L.stage = o;
  o += al16((uint32_t)(kOPos + span + 4) * 4u);
  L.cnt = o;
  o += al16((uint32_t)(kOW * cw) * 4u);
  L.tsum = o;
  o += al16((uint32_t)c * nb * kOT * 4u);
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
                            : reinterpret_cast<const float*>(a.b);
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

template <int NB>
__global__ void __launch_bounds__(kOT) pass1_owner_kernel(Pass1Args a, int vec_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int CMAX = NB == 2 ? kOColsNB2 : kOColsNB1;
  const int c0 = blockIdx.y * a.c;
  const int cs = min(a.c, a.q - c0);
  const int blo = blockIdx.z * a.bucket_span;
  const int span = min(a.bucket_span, a.r1 - blo);
  const int cw = NB == 2 ? (span + 1) >> 1 : span;  // counter words per wave
  const OwnLayout Ly = own_layout(a.bucket_span, a.c);
  float* stage = reinterpret_cast<float*>(smem + Ly.stage);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem + Ly.cnt);
  float* tsum = reinterpret_cast<float*>(smem + Ly.tsum);
  uint32_t* sgn = reinterpret_cast<uint32_t*>(smem + Ly.sgn);
  uint32_t* wsum = reinterpret_cast<uint32_t*>(smem + Ly.wsum);
  const uint32_t trash = (uint32_t)(kOPos + span) * 4u;  // discard slot (bucket outside the range)

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, L = lane & 15;
  const bool vok = vec_ok != 0;
  const int log2s = a.log2s;
  const float scale_h = a.scale_h;
  uint32_t* mycnt = cnt + wave * cw;

  double m[NB][CMAX];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int cc = 0; cc < CMAX; ++cc) m[u][cc] = 0.0;

  const int64_t row0 = (int64_t)blockIdx.x * a.rows_per_range;
  const int64_t tiles_end = (a.n_pad + kOTile - 1) / kOTile * kOTile;
  const int64_t row1 = min(tiles_end, row0 + a.rows_per_range);

  float v[16], vn[16], cI[16], cH[16];
  uint32_t sm[16], slI[16], slH[16];

  for (int64_t tile = row0; tile < row1; tile += kOTile) {
    const int64_t tl = tile + (int64_t)wave * kORowsWave;  // window-local first row of this wave
    const uint64_t jg0 = (uint64_t)a.row0g + (uint64_t)tl;  // its global row
    own_load(a, c0, tl, lane, vok, vn);                     // column 0, in flight during set-up

    // ---- set-up of the tile (independent of X) ----
    for (int i = tid; i < kOW * cw; i += kOT) cnt[i] = 0u;
    if (a.sign_flip && lane < 8) {
      const uint4 sw = stream_words(a.seed, kStreamSign, (jg0 >> 7) + (uint64_t)lane, a.instance);
      *reinterpret_cast<uint4*>(&sgn[wave * 32 + 4 * lane]) = sw;
    }
    // Bucket and Cauchy of the 32 positions, one pair of rows per step: the
    // I-half copies, then the H-half ones, each half through this thread's
    // 16 slots of the staging array (unused until the columns start), so that
    // only one step's values are live at a time.
    {
      uint2* scr = reinterpret_cast<uint2*>(stage);
      int lane_o = lane;
      asm volatile("" : "+v"(lane_o));  // keeps the per-lane row offsets inside the tile loop
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
#pragma unroll 1
        for (int g = 0; g < 8; ++g) {
          const int k = g >> 1, p = g & 1, r = 4 * k + 2 * p;
          const uint64_t j = jg0 + (uint64_t)(hh ? span_row_out(lane_o, r, log2s)
                                                  : 2 * p + 4 * lane_o + 256 * k);
          const uint64_t pos = h_position(j, log2s) + (hh ? 0ull : (1ull << log2s));
          const uint4 w = stream_words(a.seed, kStreamPi1, pos >> 1, a.instance);
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

    // ranks within (wave, bucket), from the counter adds
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint32_t& key = h ? slH[r] : slI[r];
        if (key != 0xFFFFFFFFu) {
          const uint32_t lb = key >> 16;
          uint32_t rank;
          if (NB == 2) {
            const uint32_t sh = (lb & 1u) * 16u;
            rank = (atomicAdd(&mycnt[lb >> 1], 1u << sh) >> sh) & 0xFFFFu;
          } else {
            rank = atomicAdd(&mycnt[lb], 1u);
          }
          key |= rank;
        }
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
          const uint32_t cv = cnt[w * cw + tid];
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
        if (tot[u] & 1u) stage[base + tot[u]] = 0.0f;  // pad the segment with a zero
        base += padded[u];
      }
      if (tid < cw) {
        uint32_t run[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) run[u] = seg0[u];
#pragma unroll
        for (int w = 0; w < kOW; ++w) {
          const uint32_t cv = cnt[w * cw + tid];
          if (NB == 2) {
            cnt[w * cw + tid] = run[0] | (run[NB - 1] << 16);
            run[0] += cv & 0xFFFFu;
            run[NB - 1] += cv >> 16;
          } else {
            cnt[w * cw + tid] = run[0];
            run[0] += cv;
          }
        }
      }
    }
    __syncthreads();  // offsets complete
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        uint32_t& key = h ? slH[r] : slI[r];
        if (key != 0xFFFFFFFFu) {
          const uint32_t lb = key >> 16;
          uint32_t off;
          if (NB == 2) off = (mycnt[lb >> 1] >> ((lb & 1u) * 16u)) & 0xFFFFu;
          else off = mycnt[lb];
          key = (off + (key & 0xFFFFu)) * 4u;
        } else {
          key = trash;
        }
      }

    // ---- the slice's columns ----
    for (int col = 0; col < cs; ++col) {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = vn[r];
      if (col + 1 < cs) own_load(a, c0 + col + 1, tl, lane, vok, vn);
      const uint32_t negb = (a.b && c0 + col == a.d) ? 0x80000000u : 0u;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        v[r] = __uint_as_float(__float_as_uint(v[r]) ^ sm[r] ^ negb);
        *reinterpret_cast<float*>(smem + Ly.stage + slI[r]) = cI[r] * v[r];
      }
      fwht_span1024(v, L, log2s);
#pragma unroll
      for (int r = 0; r < 16; ++r) *reinterpret_cast<float*>(smem + Ly.stage + slH[r]) = cH[r] * v[r];
      __syncthreads();  // the column's staging array is complete
      float sacc[NB];
      const float2* st2 = reinterpret_cast<const float2*>(stage);
      if (span >= 256) {
        // about 2 * 8192 / span <= 64 terms per segment: FP32 is within 64 u
        // of the segment's l1 mass
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          float sv = 0.0f;
#pragma unroll 4
          for (uint32_t q2 = seg0[u] >> 1; q2 < (seg1[u] >> 1); ++q2) {
            const float2 x = st2[q2];
            sv += x.x;
            sv += x.y;
          }
          sacc[u] = sv;
        }
      } else {
        // long segments (few buckets): sum in FP64
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          double sv = 0.0;
#pragma unroll 4
          for (uint32_t q2 = seg0[u] >> 1; q2 < (seg1[u] >> 1); ++q2) {
            const float2 x = st2[q2];
            sv += (double)x.x;
            sv += (double)x.y;
          }
          sacc[u] = (float)sv;
        }
      }
      if (NB == 2)
        reinterpret_cast<float2*>(tsum)[col * kOT + tid] = make_float2(sacc[0], sacc[NB - 1]);
      else
        tsum[col * kOT + tid] = sacc[0];
      __syncthreads();  // the staging array is rewritten by the next column
    }
    // parked per-column sums into the FP64 accumulators (written by this thread)
#pragma unroll
    for (int cc = 0; cc < CMAX; ++cc)
      if (cc < cs) {
        if (NB == 2) {
          const float2 x = reinterpret_cast<const float2*>(tsum)[cc * kOT + tid];
          m[0][cc] += (double)x.x;
          m[NB - 1][cc] += (double)x.y;
        } else {
          m[0][cc] += (double)tsum[cc * kOT + tid];
        }
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
        if (bkt < span) dst[bkt] = (float)m[u][cc];
      }
    }
}

int pass1_owner_max_cols(int span) {
  const int nb = span > 512 ? 2 : 1;
  const int cap = nb == 2 ? kOColsNB2 : kOColsNB1;
  int c = cap;
  while (c > 1 && own_layout(span, c).total > 160u * 1024u) --c;
  return c;
}

size_t pass1_owner_lds(int span, int c) { return own_layout(span, c).total; }

int pass1_owner_tile_rows() { return kOTile; }

hipError_t launch_pass1_owner(const Pass1Args& a, const Pass1Plan& p, bool vec_ok, hipStream_t st) {
  const bool two = a.bucket_span > 512;
  const void* fn = two ? (const void*)pass1_owner_kernel<2> : (const void*)pass1_owner_kernel<1>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
  if (e != hipSuccess) return e;
  const dim3 grid(p.nranges, p.nslices, p.nbranges);
  if (two)
    hipLaunchKernelGGL(pass1_owner_kernel<2>, grid, dim3(kOT), p.lds, st, a, vec_ok ? 1 : 0);
  else
    hipLaunchKernelGGL(pass1_owner_kernel<1>, grid, dim3(kOT), p.lds, st, a, vec_ok ? 1 : 0);
  return hipGetLastError();
}

}  // namespace fctl1
