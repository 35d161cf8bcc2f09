// FP64 QR of the sketch Pi1 X (r1 x q) and M = R^-1 Pi2.
//
// FastL1Basis figure / regression figure step 2: Pi1 X = Q R; only R is
// needed (U = X R^-1 is never formed; step 4 uses X (R^-1 Pi2)).  The
// running-time paragraph of the regression proof costs this O(r1 q^2).
//
// The tall factorization is a reduction tree: each workgroup factors a panel
// of P rows held in LDS with Householder reflections and emits its q x q R;
// the stacked R's form the next level's input until one panel remains.  R of
// a stack of R's equals R of the original rows up to row signs, which the
// last step fixes (positive diagonal, the unique R of a full-rank matrix).
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

static constexpr int kQrThreads = 1024;
static constexpr int kQrLdsDoubles = 16000;  // 125 KB panel budget

static int qr_panel_rows(int q) { return kQrLdsDoubles / q; }

__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// Householder QR of rows [p P, p P + m) of In (m_total x q, ld = ldin);
// writes the q x q upper R into rows [p q, p q + q) of Out (ld = ldout).
__global__ void __launch_bounds__(kQrThreads) qr_panel_kernel(const double* __restrict__ In,
                                                              int64_t m_total, int q, int64_t ldin,
                                                              int P, double* __restrict__ Out,
                                                              int64_t ldout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Pm = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[kQrThreads / 64];
  __shared__ double wdot[128];
  __shared__ double sh_beta, sh_rkk, sh_sigma;
  const int p = blockIdx.x;
  const int64_t r0 = (int64_t)p * P;
  const int m = (int)min((int64_t)P, m_total - r0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kQrThreads / 64;
  for (int idx = tid; idx < m * q; idx += kQrThreads) {
    const int i = idx % m, j = idx / m;
    Pm[idx] = In[r0 + i + (int64_t)j * ldin];
  }
  __syncthreads();
  const int kmax = min(m, q);
  // sigma_k = sum over rows i > k of P[i, k]^2: for column 0 from all threads;
  // for column k + 1 by wave 0 while it applies reflection k to that column
  {
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += kQrThreads) part += Pm[i] * Pm[i];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      double sigma = 0.0;
      for (int w = 0; w < nw; ++w) sigma += red[w];
      sh_sigma = sigma;
    }
  }
  for (int k = 0; k < kmax; ++k) {
    double* colk = Pm + (size_t)k * m;
    if (tid == 0) {
      // R_{k-1,k-1} replaces v_{k-1} now that reflection k - 1 is applied
      if (k > 0) Pm[(size_t)(k - 1) * m + (k - 1)] = sh_rkk;
      const double sigma = sh_sigma;
      const double alpha = colk[k];
      const double norm = sqrt(alpha * alpha + sigma);
      if (norm == 0.0) {
        sh_beta = 0.0;
        sh_rkk = 0.0;
      } else {
        const double rkk = alpha >= 0.0 ? -norm : norm;
        colk[k] = alpha - rkk;  // v_k; v_i = colk[i] below
        sh_beta = 1.0 / (norm * (norm + fabs(alpha)));
        sh_rkk = rkk;
      }
    }
    __syncthreads();
    const double beta = sh_beta;
    if (beta != 0.0) {
      // w_j = beta * v^T P[:, j] for the trailing columns (one wave per column)
      for (int j = k + 1 + wave; j < q; j += nw) {
        const double* colj = Pm + (size_t)j * m;
        double dot = 0.0;
        for (int i = k + lane; i < m; i += 64) dot += colk[i] * colj[i];
        dot = wave_sum(dot);
        if (lane == 0) wdot[j] = dot * beta;
      }
      __syncthreads();
      // P[i, j] -= v_i w_j: one wave per trailing column, lanes over rows
      for (int j = k + 1 + wave; j < q; j += nw) {
        double* colj = Pm + (size_t)j * m;
        const double wj = wdot[j];
        double part = 0.0;
        for (int i = k + lane; i < m; i += 64) {
          const double v = colj[i] - colk[i] * wj;
          colj[i] = v;
          if (i > k + 1) part += v * v;
        }
        if (j == k + 1) {  // wave 0
          part = wave_sum(part);
          if (lane == 0) sh_sigma = part;
        }
      }
    } else if (wave == 0 && k + 1 < q) {
      const double* colj = Pm + (size_t)(k + 1) * m;
      double part = 0.0;
      for (int i = k + 2 + lane; i < m; i += 64) part += colj[i] * colj[i];
      part = wave_sum(part);
      if (lane == 0) sh_sigma = part;
    }
    __syncthreads();
  }
  if (tid == 0 && kmax > 0) Pm[(size_t)(kmax - 1) * m + (kmax - 1)] = sh_rkk;
  __syncthreads();
  for (int idx = tid; idx < q * q; idx += kQrThreads) {
    const int i = idx % q, j = idx / q;
    const double v = (i <= j && i < m) ? Pm[i + (size_t)j * m] : 0.0;
    Out[(int64_t)p * q + i + (int64_t)j * ldout] = v;
  }
}

// Last step: positive diagonal, rank check, R (q x q, ld = q).  Column j of
// the sketch has norm ||R[:, j]||_2 (Q has orthonormal columns) and |R_jj| is
// the norm of its component orthogonal to the earlier columns.
__global__ void qr_finish_kernel(const double* __restrict__ Rin, int64_t ldin, int q,
                                 double rank_tol, double* __restrict__ R,
                                 int* __restrict__ status) {
  const int tid = threadIdx.x;
  for (int j = tid; j < q; j += blockDim.x) {
    double nrm2 = 0.0;
    for (int i = 0; i <= j; ++i) {
      const double v = Rin[i + (int64_t)j * ldin];
      nrm2 += v * v;
    }
    const double djj = fabs(Rin[j + (int64_t)j * ldin]);
    if (!isfinite(nrm2) || !(djj > rank_tol * sqrt(nrm2))) *status = -4;
  }
  for (int idx = tid; idx < q * q; idx += blockDim.x) {
    const int i = idx % q, j = idx / q;
    const double di = Rin[i + (int64_t)i * ldin];
    const double v = (i <= j) ? Rin[i + (int64_t)j * ldin] : 0.0;
    R[i + (int64_t)j * q] = di < 0.0 ? -v : v;
  }
}

static hipError_t launch_qr_panel(const double* in, int64_t m, int q, int64_t ldin, int P,
                                  double* out, int64_t np, hipStream_t st) {
  const int prow = (int)(m < P ? m : P);
  const size_t lds = (size_t)prow * q * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)qr_panel_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(qr_panel_kernel, dim3((unsigned)np), dim3(kQrThreads), lds, st, in, m, q,
                     ldin, P, out, np * q);
  return hipGetLastError();
}

size_t qr_work_doubles(int r1, int q) {
  const int P = qr_panel_rows(q);
  size_t tot = 0;
  int64_t m = r1;
  while (m > P) {
    const int64_t np = (m + P - 1) / P;
    tot += (size_t)np * q * q;
    m = np * q;
  }
  return tot + (size_t)q * q;
}

hipError_t launch_qr(const double* Y, int r1, int q, double* work, double* R, double rank_tol,
                     int* status, hipStream_t st) {
  const int P = qr_panel_rows(q);
  if (P < 2 * q) return hipErrorInvalidValue;
  const double* in = Y;
  int64_t m = r1, ldin = r1;
  double* out = work;
  hipError_t e;
  while (true) {
    const int64_t np = (m + P - 1) / P;
    e = launch_qr_panel(in, m, q, ldin, P, out, np, st);
    if (e != hipSuccess) return e;
    if (np == 1) break;
    in = out;
    ldin = np * q;
    m = np * q;
    out += (size_t)np * q * q;
  }
  hipLaunchKernelGGL(qr_finish_kernel, dim3(1), dim3(256), 0, st, out, (int64_t)q, q, rank_tol, R,
                     status);
  return hipGetLastError();
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// M = R^-1 Pi2: Pi2 is drawn by all threads into LDS, then one thread per
// column of Pi2 back-substitutes against R held in LDS.
__global__ void __launch_bounds__(256) form_m_kernel(const double* __restrict__ R, int q, int r2,
                                                     int ldm, uint64_t seed, uint32_t instance,
                                                     double* __restrict__ Md, float* __restrict__ Mf,
                                                     float* __restrict__ Mfb,
                                                     uint16_t* __restrict__ Mb,
                                                     int* __restrict__ status, int gaussian) {
  __shared__ double Rs[96 * 96];
  __shared__ double Ms[96 * 32];
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) Rs[e] = R[e];
  for (int e = threadIdx.x; e < q * ldm; e += blockDim.x) {
    const int a = e / ldm, c = e % ldm;
    double v = 0.0;
    if (c < r2) {
      const uint4 w = stream_words(seed, kStreamPi2, (uint64_t)a * r2 + c, instance);
      v = gaussian ? gaussian_from_words_f64(w.x, w.y) : cauchy_from_word_f64(w.x);
    }
    Ms[e] = v;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < r2) {
    for (int a = q - 1; a >= 0; --a) {
      double v = Ms[a * ldm + c];
      for (int bcol = a + 1; bcol < q; ++bcol) v -= Rs[a + bcol * q] * Ms[bcol * ldm + c];
      v = v / Rs[a + a * q];
      if (!isfinite(v)) *status = -4;
      Ms[a * ldm + c] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < q * ldm; e += blockDim.x) {
    const double v = Ms[e];
    const float f = (float)v;
    const uint16_t h = f32_to_bf16_rne(f);
    Md[e] = v;
    if (Mf) Mf[e] = f;
    if (Mfb) Mfb[e] = __uint_as_float((uint32_t)h << 16);
    if (Mb) Mb[e] = h;
  }
}

hipError_t launch_form_m(const double* R, int q, int r2, int ldm, uint64_t seed,
                         uint32_t instance, double* Md, float* Mf, float* Mfb, uint16_t* Mb,
                         int* status, hipStream_t st, bool gaussian) {
  if (q > 96 || ldm > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(form_m_kernel, dim3(1), dim3(256), 0, st, R, q, r2, ldm, seed, instance, Md,
                     Mf, Mfb, Mb, status, gaussian ? 1 : 0);
  return hipGetLastError();
}

}  // namespace fctl1
