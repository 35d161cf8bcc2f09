// Step 8 of the regression figure: x_hat = argmin ||D A x - D b||_1 on the
// coreset, i.e. min_x sum_k w_k |a_k^T x - b_k| with w_k = 1/p_k.  The paper
// solves it by linear programming; here it is solved in FP64 on the GPU by
// iteratively reweighted least squares on the smoothed objective
// sum_k w_k sqrt(r_k^2 + eta^2) (each step minimizes the quadratic majorant
// sum_k w_k r_k^2 / sqrt(r_k^2 + eta^2), so the smoothed objective never
// increases), with eta shrunk by 5x per step to a floor; the smoothed and
// the exact objective differ by at most eta sum_k w_k.  The floor is 1e-6 of the
// mean weighted residual, so the smoothing costs at most 1e-6 of the
// objective: smaller floors give weights so uneven that FP64 rounding in the
// Gram matrix makes the iterates wander.  The result is the iterate with the
// lowest exact objective seen; at the floor the iteration stops once the
// objective moves by at most 1e-9 relatively or has not improved three times.
//
// The whole iteration is one persistent cooperative kernel.  Each workgroup
// owns a contiguous range of coreset rows and, per iteration, accumulates the
// weighted Gram matrix of [A b] over its rows in 4x4 register blocks (FP64),
// writes it as a partial, and meets the others at a grid barrier.  Every
// workgroup then sums all partials in the same fixed order and runs the same
// Gauss-Jordan solve, so all of them hold bit-identical x, objective and
// stopping decision without a second barrier.  Partials are double-buffered by
// iteration parity: a workgroup can run at most one iteration ahead.
#include "fct_device.h"
#include "fct_kernels.h"

#include <cstdlib>

namespace fctl1 {

static constexpr int kIrlsThreads = 256;
static constexpr int kIrlsMaxD = 64;
static constexpr int kIrlsMaxWgs = 64;
static constexpr int kIrlsRowTarget = 320;  // coreset rows per workgroup the grid is sized for
static constexpr size_t kIrlsLdsBytes = 150 * 1024;
static constexpr int kGjMax = (64 * 65 + 255) / 256;  // augmented entries per thread, d = 64
static constexpr unsigned kSpinLimit = 1u << 24;  // polls of ~64 clocks each before giving up

// Geometry of the augmented Gram [A b]^T W [A b] in 4x4 blocks, and the LDS
// plan: resident rows (element type T) + one weight per row, then the Gram
// area (also the per-group partial sums before the barrier) and vectors.
struct IrlsGeom {
  int d, q, NB, W, nbp, groups, pstride, E;
  size_t gdoubles, fixed_bytes;
  __host__ __device__ IrlsGeom(int d_, size_t elem) {
    d = d_;
    q = d + 1;
    NB = (q + 3) / 4;
    W = 4 * NB;
    nbp = NB * (NB + 1) / 2;
    groups = kIrlsThreads / nbp;
    if (groups < 1) groups = 1;
    E = nbp * 16 + 1;
    pstride = (E + 7) & ~7;
    const size_t g1 = (size_t)d * d, g2 = (size_t)groups * nbp * 16;
    gdoubles = ((g1 > g2 ? g1 : g2) + 1) & ~(size_t)1;  // keeps the vectors 16-byte aligned
    fixed_bytes = (((gdoubles + 64 + 72 + 80 + 16 + 512 + 528 + 264 + 64 + 256 + 64) * sizeof(double)) + 15) &
                  ~(size_t)15;
    row_bytes = (size_t)W * elem + sizeof(double);
    rmax = (int)((kIrlsLdsBytes - fixed_bytes) / row_bytes);
    rmax &= ~63;
  }
  size_t row_bytes;
  int rmax;  // rows a workgroup holds in LDS at once
  __host__ __device__ size_t lds_bytes() const { return fixed_bytes + (size_t)rmax * row_bytes; }
};


size_t irls_work_doubles(int64_t S, int d) {
  (void)S;
  const IrlsGeom g(d, sizeof(double));
  return 2 * (size_t)kIrlsMaxWgs * g.pstride + 8;
}

// Grid-wide barrier on a monotone arrival counter.  The agent-scope fences
// publish this workgroup's partial stores before its arrival and make the
// others' visible after the wait.  The wait is bounded: on timeout the abort
// flag is raised so every workgroup leaves at its next barrier.
__device__ bool grid_barrier(unsigned* bar, unsigned target, int* ok_sh) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          ++spins > kSpinLimit) {
        __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *ok_sh = ok;
  }
  __syncthreads();
  __threadfence();
  return *ok_sh != 0;
}

__device__ inline void block_pair(int pr, int NB, int& bi, int& bj) {
  int i = 0, rem = pr;
  while (rem >= NB - i) {
    rem -= NB - i;
    ++i;
  }
  bi = i;
  bj = i + rem;
}

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps.
__device__ inline double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

template <typename T>
__device__ inline void load4(const T* p, double (&v)[4]);
template <>
__device__ inline void load4<float>(const float* p, double (&v)[4]) {
  const float4 f = *reinterpret_cast<const float4*>(p);
  v[0] = f.x;
  v[1] = f.y;
  v[2] = f.z;
  v[3] = f.w;
}
template <>
__device__ inline void load4<double>(const double* p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

// Inverse of a 4x4 symmetric positive definite block (row-major in, out) by
// its Cholesky factor: D^-1 = L^-T L^-1.  Returns false if a pivot of the
// factorization is not positive.
__device__ inline bool spd4_inverse(const double* a, double* inv) {
  const double r0 = rsqrt_f64(fmax(a[0], 1e-300));
  const double l10 = a[4] * r0, l20 = a[8] * r0, l30 = a[12] * r0;
  const double p1 = a[5] - l10 * l10;
  const double r1 = rsqrt_f64(fmax(p1, 1e-300));
  const double l21 = (a[9] - l20 * l10) * r1, l31 = (a[13] - l30 * l10) * r1;
  const double p2 = a[10] - l20 * l20 - l21 * l21;
  const double r2 = rsqrt_f64(fmax(p2, 1e-300));
  const double l32 = (a[14] - l30 * l20 - l31 * l21) * r2;
  const double p3 = a[15] - l30 * l30 - l31 * l31 - l32 * l32;
  const double r3 = rsqrt_f64(fmax(p3, 1e-300));
  // M = L^-1 (lower): diagonal r_i
  const double m10 = -l10 * r0 * r1;
  const double m21 = -l21 * r1 * r2;
  const double m20 = -(l20 * r0 + l21 * m10) * r2;
  const double m32 = -l32 * r2 * r3;
  const double m31 = -(l31 * r1 + l32 * m21) * r3;
  const double m30 = -(l30 * r0 + l31 * m10 + l32 * m20) * r3;
  // D^-1 = M^T M
  inv[0] = r0 * r0 + m10 * m10 + m20 * m20 + m30 * m30;
  inv[1] = m10 * r1 + m20 * m21 + m30 * m31;
  inv[2] = m20 * r2 + m30 * m32;
  inv[3] = m30 * r3;
  inv[5] = r1 * r1 + m21 * m21 + m31 * m31;
  inv[6] = m21 * r2 + m31 * m32;
  inv[7] = m31 * r3;
  inv[10] = r2 * r2 + m32 * m32;
  inv[11] = m32 * r3;
  inv[15] = r3 * r3;
  inv[4] = inv[1];
  inv[8] = inv[2];
  inv[9] = inv[6];
  inv[12] = inv[3];
  inv[13] = inv[7];
  inv[14] = inv[11];
  return a[0] > 1e-15 && p1 > 1e-15 && p2 > 1e-15 && p3 > 1e-15;
}

// Block Gauss-Jordan on the Jacobi-scaled augmented system
// [S G S | S rhs] (n4 x (n4 + 1), identity rows and columns pad d to n4, a
// multiple of 4), all threads of the workgroup; thread tid keeps entries
// (er[u], ec[u]), u < NE, in registers.  Step K publishes the pivot block's
// columns and rows (double-buffered by step parity), forms T = D^-1 (pivot
// rows) with D the 4x4 pivot block, then pivot rows become T and every other
// row r loses M[r, P] T.  The last column ends as z with (S G S) z = S rhs;
// it is written to z[0..d).  Returns false if a pivot block is not positive
// definite.
template <int NE>
__device__ __forceinline__ bool gj_solve(const int* er, const int* ec, const double* G,
                                         const double* rhs, const double* sc, double* gjcol2,
                                         double* gjrow2, double* gjt, double* gjd, int d,
                                         double* z) {
  const int tid = threadIdx.x;
  const int n4 = (d + 3) & ~3, nc = n4 + 1;
  double mv[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int r = er[u], c = ec[u];
    double v = 0.0;
    if (r >= 0) {
      if (c == n4) v = r < d ? rhs[r] * sc[r] : 0.0;
      else if (r < d && c < d) v = G[r * d + c] * sc[r] * sc[c];
      else v = r == c ? 1.0 : 0.0;
    }
    mv[u] = v;
  }
  double* dummy = gjd + tid;
  bool ok = true;
  for (int K = 0; K < n4 / 4; ++K) {
    const int p0 = 4 * K;
    double* gjcol = gjcol2 + (K & 1) * 256;  // gjcol[r][m] = M[r][p0 + m]
    double* gjrow = gjrow2 + (K & 1) * 264;  // gjrow[c][m] = M[p0 + m][c]
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int r = er[u], c = ec[u];
      const bool inc = r >= 0 && (unsigned)(c - p0) < 4u;
      const bool inr = r >= 0 && (unsigned)(r - p0) < 4u;
      *(inc ? gjcol + r * 4 + (c - p0) : dummy) = mv[u];
      *(inr ? gjrow + c * 4 + (r - p0) : dummy) = mv[u];
    }
    __syncthreads();
    if (tid < nc) {
      double Dm[16], Di[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) Dm[e] = gjcol[(p0 + (e >> 2)) * 4 + (e & 3)];
      ok = spd4_inverse(Dm, Di) && ok;
      const double2 q01 = *reinterpret_cast<const double2*>(gjrow + tid * 4);
      const double2 q23 = *reinterpret_cast<const double2*>(gjrow + tid * 4 + 2);
#pragma unroll
      for (int m = 0; m < 4; ++m)
        gjt[tid * 4 + m] = Di[4 * m] * q01.x + Di[4 * m + 1] * q01.y + Di[4 * m + 2] * q23.x +
                           Di[4 * m + 3] * q23.y;
    }
    __syncthreads();
    // loads of a chunk of entries are issued together, then their updates
    constexpr int CH = NE < 5 ? NE : 5;
#pragma unroll
    for (int u0 = 0; u0 < NE; u0 += CH) {
      double2 t01[CH], t23[CH], a01[CH], a23[CH];
#pragma unroll
      for (int v = 0; v < CH; ++v) {
        const int u = u0 + v < NE ? u0 + v : NE - 1;
        const int r = er[u] >= 0 ? er[u] : 0, c = ec[u];
        t01[v] = *reinterpret_cast<const double2*>(gjt + c * 4);
        t23[v] = *reinterpret_cast<const double2*>(gjt + c * 4 + 2);
        a01[v] = *reinterpret_cast<const double2*>(gjcol + r * 4);
        a23[v] = *reinterpret_cast<const double2*>(gjcol + r * 4 + 2);
      }
#pragma unroll
      for (int v = 0; v < CH; ++v) {
        const int u = u0 + v;
        if (u < NE) {
          const double upd = mv[u] - (a01[v].x * t01[v].x + a01[v].y * t01[v].y +
                                      a23[v].x * t23[v].x + a23[v].y * t23[v].y);
          const int rm = er[u] - p0;
          const double tp =
              rm == 0 ? t01[v].x : rm == 1 ? t01[v].y : rm == 2 ? t23[v].x : t23[v].y;
          mv[u] = (unsigned)rm < 4u ? tp : upd;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NE; ++u)
    if (ec[u] == n4 && er[u] >= 0 && er[u] < d) z[er[u]] = mv[u];
  return ok;
}

// d > 48: kept out of line so that its register demand does not raise the
// kernel's own.
__device__ __noinline__ bool gj_solve_wide(const double* G, const double* rhs, const double* sc,
                                           double* gjcol2, double* gjrow2, double* gjt,
                                           double* gjd, int d, double* z) {
  const int n4 = (d + 3) & ~3, nc = n4 + 1;
  int er[kGjMax], ec[kGjMax];
#pragma unroll
  for (int u = 0; u < kGjMax; ++u) {
    const int e = threadIdx.x + kIrlsThreads * u;
    er[u] = e < n4 * nc ? e / nc : -1;
    ec[u] = e < n4 * nc ? e - er[u] * nc : 0;
  }
  return gj_solve<kGjMax>(er, ec, G, rhs, sc, gjcol2, gjrow2, gjt, gjd, d, z);
}

// BATCH: every instance has its own barrier word, partials and status.
// Without binst, workgroup b solves instance arr[b] alone; with it, block b
// belongs to instance binst[b] as its workgroup b - wg0 of nwg, and the
// instance's workgroups meet at its own barrier (the launch keeps the grid
// within what the device holds at once).  Otherwise the grid cooperates on
// the instance a0.
template <typename T, bool BATCH>
__global__ void __launch_bounds__(kIrlsThreads) irls_kernel(IrlsArgs a0, const IrlsArgs* __restrict__ arr,
                                                           const int* __restrict__ binst) {
  const int inst = BATCH ? (binst ? binst[blockIdx.x] : (int)blockIdx.x) : 0;
  const IrlsArgs a = BATCH ? arr[inst] : a0;
  const int wg = BATCH ? (binst ? (int)blockIdx.x - a.wg0 : 0) : (int)blockIdx.x;
  const int gcount = BATCH ? (binst ? a.nwg : 1) : (int)gridDim.x;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int flag_stop, flag_bad, flag_ok, flag_best;
  const IrlsGeom g(a.d, sizeof(T));
  const int d = g.d, q = g.q, W = g.W, NB = g.NB, nbp = g.nbp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* G = reinterpret_cast<double*>(smem);  // Gram, or group partials before the barrier
  double* rhs = G + g.gdoubles;
  double* xs = rhs + 64;    // 72: x, then -1 at d, zeros to the padded width
  double* sc = xs + 72;     // 80: d + 1 scales
  double* misc = sc + 80;   // [0] sum w, [1] eta, [2] prev obj, [3] floor, [5] obj,
                            // [6] best obj, [7] non-improving steps at the floor, [8..11] waves
  double* gjcol2 = misc + 16;    // 2 x 64 x 4: pivot columns of the Gauss-Jordan step
  double* gjrow2 = gjcol2 + 512; // 2 x 65 x 4: pivot rows, transposed
  double* gjt = gjrow2 + 528;    // 65 x 4: D^-1 times the pivot rows, transposed
  double* gjz = gjt + 264;       // 64: solution
  double* gjd = gjz + 64;        // 256: per-thread dummy slots
  double* bx = gjd + 256;        // 64: the best iterate
  double* om = reinterpret_cast<double*>(smem + g.fixed_bytes);
  T* zr = reinterpret_cast<T*>(om + g.rmax);
  const T* At = (const T*)a.At;
  const T* bt = (const T*)a.bt;
  const int64_t S = min(*a.S_dev, a.cap);
  // active workgroups: about kIrlsRowTarget rows each, never more than fit in
  // LDS unless even the whole grid cannot hold them (then rows stream through)
  int64_t pa = (S + a.row_target - 1) / a.row_target;
  const int64_t pmin = (S + g.rmax - 1) / g.rmax;
  if (pa < pmin) pa = pmin;
  if (pa > (int64_t)gcount) pa = gcount;
  if (pa < 1) pa = 1;
  const int P = (int)pa;
  if ((int)wg >= P) return;
  const int64_t per = (S + P - 1) / P;
  const int64_t lo = min(S, (int64_t)wg * per), hi = min(S, lo + per);
  const bool resident = hi - lo <= g.rmax;

  // sum of weights, in the same order in every workgroup
  double sw = 0.0;
  for (int64_t k = tid; k < S; k += kIrlsThreads) sw += a.w[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sw += __shfl_xor(sw, o, 64);
  if (lane == 0) misc[8 + wave] = sw;
  if (tid < 72) xs[tid] = tid == d ? -1.0 : 0.0;
  __syncthreads();
  if (tid == 0) {
    const double t = misc[8] + misc[9] + misc[10] + misc[11];
    misc[0] = t > 0.0 ? t : 1.0;
    misc[1] = 0.0;
    misc[2] = 0.0;
    misc[3] = 0.0;
    misc[6] = HUGE_VAL;
    misc[7] = 0.0;
  }

  // entries of the augmented n4 x (n4 + 1) system owned by this thread in the
  // Gauss-Jordan solve: e = tid + threads * u
  const int n4 = (d + 3) & ~3, nc = n4 + 1, ne = (n4 * nc + kIrlsThreads - 1) / kIrlsThreads;
  int er[10], ec[10];  // d <= 48; wider systems decode their own entries
#pragma unroll
  for (int u = 0; u < 10; ++u) {
    const int e = tid + kIrlsThreads * u;
    er[u] = -1;
    ec[u] = 0;  // absent entries read column 0 and publish to the dummy slot
    if (u < ne && e < n4 * nc) {
      er[u] = e / nc;
      ec[u] = e - er[u] * nc;
    }
  }
  // this thread's 4x4 block (bi <= bj) of the Gram and its share of the rows
  const int pair = tid % nbp, grp = tid / nbp;
  const bool gram_thread = grp < g.groups;
  int bi, bj;
  block_pair(pair, NB, bi, bj);

  for (int it = 0;; ++it) {
    __syncthreads();
    const double eta = misc[1];
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0;
    double objp = 0.0;
    for (int64_t c0 = lo; c0 < hi; c0 += g.rmax) {
      const int nr = (int)min<int64_t>(g.rmax, hi - c0);
      if (!resident || it == 0) {
        __syncthreads();
        for (int r0 = 0; r0 < nr; r0 += 64) {
          const int r = r0 + lane;
          for (int c = wave; c < W; c += 4) {
            T v = (T)0;
            if (r < nr && c < q) v = c < d ? At[c0 + r + (int64_t)c * a.ldat] : bt[c0 + r];
            zr[r * W + c] = v;
          }
        }
        __syncthreads();
      }
      // residuals at x, objective, IRLS weights
      for (int r = tid; r < nr; r += kIrlsThreads) {
        const T* z = zr + r * W;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int c = 0; c < W; c += 4) {
          double zv[4];
          load4<T>(z + c, zv);
          const double2 x01 = *reinterpret_cast<const double2*>(xs + c);
          const double2 x23 = *reinterpret_cast<const double2*>(xs + c + 2);
          s4[0] = fma(zv[0], x01.x, s4[0]);
          s4[1] = fma(zv[1], x01.y, s4[1]);
          s4[2] = fma(zv[2], x23.x, s4[2]);
          s4[3] = fma(zv[3], x23.y, s4[3]);
        }
        // xs[d] = -1 and xs[d+1..W) = 0, so the sum is a^T x - b
        const double res = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        const double wk = a.w[c0 + r];
        objp += wk * fabs(res);
        om[r] = eta > 0.0 ? wk / sqrt(res * res + eta * eta) : wk;
      }
      __syncthreads();
      if (gram_thread && grp < nr) {
        // one row ahead: the loads of row rr + groups are issued before the
        // products of row rr (the clamped index keeps them in bounds)
        double av[4], bv[4], o;
        load4<T>(zr + grp * W + 4 * bi, av);
        load4<T>(zr + grp * W + 4 * bj, bv);
        o = om[grp];
        for (int rr = grp; rr < nr; rr += g.groups) {
          const int rn = min(rr + g.groups, nr - 1);
          double an[4], bn[4];
          load4<T>(zr + rn * W + 4 * bi, an);
          load4<T>(zr + rn * W + 4 * bj, bn);
          const double on = om[rn];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double oa = o * av[i];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[4 * i + j] = fma(oa, bv[j], acc[4 * i + j]);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            av[i] = an[i];
            bv[i] = bn[i];
          }
          o = on;
        }
      }
      if (!resident) __syncthreads();
    }
    // workgroup partial: sum the row groups in order, then publish
    objp = wave_sum_dpp(objp);
    if (lane == 0) misc[8 + wave] = objp;
    if (gram_thread)
#pragma unroll
      for (int e = 0; e < 16; ++e) G[(grp * nbp + pair) * 16 + e] = acc[e];
    __syncthreads();
    double* mine = a.part + ((size_t)(it & 1) * P + wg) * g.pstride;
    for (int e = tid; e < nbp * 16; e += kIrlsThreads) {
      double s = 0.0;
      for (int gg = 0; gg < g.groups; ++gg) s += G[gg * nbp * 16 + e];
      mine[e] = s;
    }
    if (tid == 0) mine[nbp * 16] = misc[8] + misc[9] + misc[10] + misc[11];
    if (!grid_barrier(a.bar, (unsigned)(it + 1) * (unsigned)P, &flag_ok)) {
      if (wg == 0 && tid == 0) *a.status = -5;
      break;
    }
    // all partials, fixed order, into the symmetric G and rhs; the loads of up
    // to four entries x sixteen partials are issued before any is summed
    const double* pb = a.part + (size_t)(it & 1) * P * g.pstride;
    for (int e0 = tid; e0 < g.E; e0 += 4 * kIrlsThreads) {
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      for (int p0 = 0; p0 < P; p0 += 16) {
        double v[4][16];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int e = e0 + k * kIrlsThreads, p = p0 + u;
            v[k][u] = (e < g.E && p < P) ? pb[(size_t)p * g.pstride + e] : 0.0;
          }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < 16; ++u) s[k] += v[k][u];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = e0 + k * kIrlsThreads;
        if (e >= g.E) continue;
        if (e == g.E - 1) {
          misc[5] = s[k];
          continue;
        }
        int pbi, pbj;
        block_pair(e >> 4, NB, pbi, pbj);
        const int ii = (e >> 2) & 3, jj = e & 3;
        if (pbi == pbj && ii > jj) continue;
        const int row = 4 * pbi + ii, col = 4 * pbj + jj;
        if (row < d && col < d) {
          G[row * d + col] = s[k];
          G[col * d + row] = s[k];
        } else if (row < d && col == d) {
          rhs[row] = s[k];
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double obj = misc[5];
      double e_c = misc[1];
      const double floor_now = 1e-6 * obj / misc[0];
      const bool at_floor = e_c > 0.0 && e_c <= misc[3] * 1.0000001;
      int stop = 0;
      const int best = obj < misc[6];  // false for a non-finite objective
      if (best) {
        misc[6] = obj;
        misc[7] = 0.0;
      } else if (at_floor) {
        misc[7] += 1.0;
      }
      if (e_c <= 0.0) {
        e_c = obj / misc[0];  // first smoothing level: mean weighted residual
      } else {
        if (at_floor && (fabs(misc[2] - obj) <= 1e-9 * obj || misc[7] >= 3.0)) stop = 1;
        e_c = fmax(floor_now, 0.2 * e_c);
      }
      if (!(obj > 0.0) || it >= a.iters) stop = 1;  // exact fit, non-finite, or budget spent
      misc[3] = floor_now;
      misc[2] = obj;
      misc[1] = e_c;
      flag_stop = stop;
      flag_best = best;
      flag_bad = 0;
    }
    __syncthreads();
    if (flag_best && tid < d) bx[tid] = xs[tid];
    if (flag_stop) break;
    // Jacobi equilibration S = diag(G)^-1/2, then block Gauss-Jordan on the
    // augmented n4 x (n4 + 1) system [S G S | S rhs] (identity rows and
    // columns pad d to n4, a multiple of 4).  Thread tid keeps entries
    // e = tid + threads * u in registers.  Step K: the pivot block's columns
    // and rows are published to LDS; D^-1 of the 4x4 pivot block gives
    // T = D^-1 (pivot rows); pivot rows become T and every other row r loses
    // M[r, P] T.  After the last step the last column holds z, x = S z.
    if (tid < d) {
      const double gg = G[tid * d + tid];
      sc[tid] = gg > 0.0 ? rsqrt_f64(gg) : 1.0;
    }
    __syncthreads();
    {
      bool ok;
      if (ne <= 2) ok = gj_solve<2>(er, ec, G, rhs, sc, gjcol2, gjrow2, gjt, gjd, d, gjz);
      else if (ne <= 5) ok = gj_solve<5>(er, ec, G, rhs, sc, gjcol2, gjrow2, gjt, gjd, d, gjz);
      else if (ne <= 10) ok = gj_solve<10>(er, ec, G, rhs, sc, gjcol2, gjrow2, gjt, gjd, d, gjz);
      else ok = gj_solve_wide(G, rhs, sc, gjcol2, gjrow2, gjt, gjd, d, gjz);
      if (!ok) flag_bad = 1;
      __syncthreads();
      if (!flag_bad && tid < d) xs[tid] = gjz[tid] * sc[tid];
    }
    __syncthreads();
    if (flag_bad) {
      // The first system carries only the coreset weights: a failed pivot
      // there means the coreset is singular.  Later systems are reweighted
      // by 1/sqrt(r^2 + eta^2), whose spread near the optimum can push a
      // Schur pivot of a full-rank coreset below the threshold; the best
      // iterate so far is then the result.
      if (it == 0 && wg == 0 && tid == 0) *a.status = -4;
      break;
    }
  }
  __syncthreads();
  if (wg == 0) {
    // the best iterate; before any objective was formed (a failed barrier on
    // the first step) that is the starting point x = 0
    const bool any = misc[6] < HUGE_VAL;
    if (tid < d) a.x_out[tid] = any ? bx[tid] : 0.0;
    if (tid == 0 && a.obj_out) *a.obj_out = any ? misc[6] : misc[2];
  }
}

__global__ void irls_reset_kernel(unsigned* bar) {
  if (threadIdx.x < 2) bar[threadIdx.x] = 0u;
}

__global__ void irls_reset_batched_kernel(const IrlsArgs* __restrict__ arr, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    arr[i].bar[0] = 0u;
    arr[i].bar[1] = 0u;
    *arr[i].status = 0;
  }
}

size_t irls_batched_work_doubles(int d, int nwg) {
  const IrlsGeom g(d, sizeof(double));
  return 2 * (size_t)nwg * g.pstride + 8;
}

unsigned* irls_batched_bar(double* work, int d, int nwg) {
  return reinterpret_cast<unsigned*>(work + irls_batched_work_doubles(d, nwg) - 8);
}

int irls_max_resident_wgs(int cus) {
  int per = 0;
  const void* fn = (const void*)irls_kernel<float, true>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kIrlsLdsBytes) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kIrlsThreads, kIrlsLdsBytes) != hipSuccess)
    return 0;
  return per * cus;
}

hipError_t launch_irls_batched(const IrlsArgs* arr, int count, bool f64, hipStream_t st,
                               const int* binst, int nblocks, bool reset) {
  if (count <= 0) return hipSuccess;
  const size_t lds = kIrlsLdsBytes;
  const void* fn = f64 ? (const void*)irls_kernel<double, true> : (const void*)irls_kernel<float, true>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  IrlsArgs none{};
  if (reset)
    hipLaunchKernelGGL(irls_reset_batched_kernel, dim3((count + 63) / 64), dim3(64), 0, st, arr, count);
  const int grid = binst ? nblocks : count;
  if (grid <= 0) return hipGetLastError();
  if (f64)
    hipLaunchKernelGGL((irls_kernel<double, true>), dim3(grid), dim3(kIrlsThreads), lds, st, none, arr, binst);
  else
    hipLaunchKernelGGL((irls_kernel<float, true>), dim3(grid), dim3(kIrlsThreads), lds, st, none, arr, binst);
  return hipGetLastError();
}

static int irls_row_target(int rows_override) {
  const int r = rows_override > 0 ? rows_override : kIrlsRowTarget;
  return r < 16 ? 16 : r;
}

static int irls_workgroups(int64_t S_hint, int rows_override, int wgs_override) {
  const int rt = irls_row_target(rows_override);
  int64_t p = wgs_override > 0 ? wgs_override : (S_hint + rt - 1) / rt;
  if (p < 1) p = 1;
  if (p > kIrlsMaxWgs) p = kIrlsMaxWgs;
  return (int)p;
}

hipError_t launch_irls(const void* At, const void* bt, const double* w, const int64_t* S_dev,
                       int64_t cap, int64_t S_hint, int d, int64_t ldat, bool f64, int iters,
                       double* work, double* x_out, double* obj_out, int* status,
                       hipStream_t st, int rows_override, int wgs_override) {
  if (d > kIrlsMaxD || d < 1) return hipErrorInvalidValue;
  const IrlsGeom g(d, f64 ? sizeof(double) : sizeof(float));
  const int P = irls_workgroups(S_hint, rows_override, wgs_override);
  IrlsArgs a;
  a.At = At;
  a.bt = bt;
  a.w = w;
  a.S_dev = S_dev;
  a.cap = cap;
  a.ldat = ldat;
  a.d = d;
  a.iters = iters;
  a.row_target = irls_row_target(rows_override);
  a.part = work;
  a.bar = reinterpret_cast<unsigned*>(work + irls_work_doubles(0, d) - 8);
  a.x_out = x_out;
  a.obj_out = obj_out;
  a.status = status;
  const size_t lds = g.lds_bytes();
  const void* fn = f64 ? (const void*)irls_kernel<double, false> : (const void*)irls_kernel<float, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(irls_reset_kernel, dim3(1), dim3(64), 0, st, a.bar);
  const IrlsArgs* none = nullptr;
  const int* nomap = nullptr;
  void* args[] = {&a, &none, &nomap};
  return hipLaunchCooperativeKernel(fn, dim3(P), dim3(kIrlsThreads), args, (unsigned)lds, st);
}

}  // namespace fctl1
