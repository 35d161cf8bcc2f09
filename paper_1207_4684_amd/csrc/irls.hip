// Step 8 of the regression figure: x_hat = argmin ||D A x - D b||_1 on the
// coreset, i.e. min_x sum_k w_k |a_k^T x - b_k| with w_k = 1/p_k.  The paper
// solves it by linear programming; here it is solved in FP64 on the GPU by
// iteratively reweighted least squares on the smoothed objective
// sum_k w_k sqrt(r_k^2 + eta^2) (each step minimizes the quadratic majorant
// sum_k w_k r_k^2 / sqrt(r_k^2 + eta^2), so the smoothed objective never
// increases), with eta decreased geometrically to a floor; the smoothed and
// the exact objective differ by at most eta sum_k w_k.
//
// Each iteration is two kernels: many workgroups accumulate partial weighted
// Gram matrices A^T W A and right-hand sides A^T W b (and the objective at the
// current x); one workgroup sums the partials in a fixed order and solves the
// normal equations by Cholesky.  A device flag ends the iteration early once
// the objective has stopped moving at the smallest eta.
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

static constexpr int kIrlsWgs = 64;
static constexpr int kIrlsThreads = 256;
static constexpr int kIrlsTile = 64;
static constexpr int kIrlsMaxD = 64;
static constexpr int kIrlsPer = (kIrlsMaxD * (kIrlsMaxD + 1) / 2 + kIrlsMaxD + kIrlsThreads - 1) / kIrlsThreads;

// work layout (doubles)
struct IrlsLayout {
  int d;
  size_t x, part, obj, state, total;
  __host__ __device__ IrlsLayout(int d_) : d(d_) {
    const size_t E = (size_t)d * d + d;
    x = 0;
    part = x + ((d + 7) & ~7);
    obj = part + (size_t)kIrlsWgs * E;
    state = obj + kIrlsWgs;
    total = state + 8;
  }
};
// state: [0] eta (<= 0: plain weighted least squares), [1] previous objective,
//        [2] done flag, [3] eta floor, [4] sum of weights, [5] last objective

size_t irls_work_doubles(int64_t S, int d) {
  (void)S;
  return IrlsLayout(d).total;
}

template <typename T>
__global__ void __launch_bounds__(kIrlsThreads) irls_gram_kernel(
    const T* __restrict__ At, const T* __restrict__ bt, const double* __restrict__ w,
    const int64_t* __restrict__ S_dev, int64_t cap, int d, int64_t ldat, double* work) {
  const IrlsLayout L(d);
  if (work[L.state + 2] != 0.0) return;
  __shared__ double xs[kIrlsMaxD];
  __shared__ double tile[kIrlsTile * (kIrlsMaxD + 1)];
  __shared__ double om[kIrlsTile];
  __shared__ double red[kIrlsThreads / 64];
  const int tid = threadIdx.x;
  const int64_t S = min(*S_dev, cap);
  const double eta = work[L.state + 0];
  for (int k = tid; k < d; k += kIrlsThreads) xs[k] = work[L.x + k];
  const int E = d * (d + 1) / 2 + d;
  // entries this thread owns: upper-triangle (i <= j) pairs, then rhs k
  double accv[kIrlsPer];
  int ei[kIrlsPer], ej[kIrlsPer];
#pragma unroll
  for (int u = 0; u < kIrlsPer; ++u) {
    accv[u] = 0.0;
    const int e = tid + u * kIrlsThreads;
    int i = 0, j = 0;
    if (e < d * (d + 1) / 2) {
      int rem = e;
      while (rem >= d - i) { rem -= d - i; ++i; }
      j = i + rem;
    } else if (e < E) {
      i = e - d * (d + 1) / 2;
      j = d;  // right-hand side entry: sum om a_i b
    }
    ei[u] = i;
    ej[u] = j;
  }
  double objp = 0.0;
  const int64_t per = (S + kIrlsWgs - 1) / kIrlsWgs;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = min(S, lo + per);
  for (int64_t t0 = lo; t0 < hi; t0 += kIrlsTile) {
    const int nt = (int)min<int64_t>(kIrlsTile, hi - t0);
    __syncthreads();
    for (int e = tid; e < nt * (d + 1); e += kIrlsThreads) {
      const int rr = e % nt, c = e / nt;
      const double v = c < d ? (double)At[t0 + rr + (int64_t)c * ldat] : (double)bt[t0 + rr];
      tile[rr * (kIrlsMaxD + 1) + c] = v;
    }
    __syncthreads();
    if (tid < nt) {
      const double* row = tile + tid * (kIrlsMaxD + 1);
      double r = -row[d];
      for (int c = 0; c < d; ++c) r = fma(row[c], xs[c], r);
      const double wk = w[t0 + tid];
      objp += wk * fabs(r);
      om[tid] = eta > 0.0 ? wk / sqrt(r * r + eta * eta) : wk;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kIrlsPer; ++u) {
      if (tid + u * kIrlsThreads < E) {
        const int i = ei[u], j = ej[u];
        double s = 0.0;
        for (int rr = 0; rr < nt; ++rr) {
          const double* row = tile + rr * (kIrlsMaxD + 1);
          s = fma(om[rr] * row[i], row[j], s);
        }
        accv[u] += s;
      }
    }
  }
  double* part = work + L.part + (size_t)blockIdx.x * ((size_t)d * d + d);
#pragma unroll
  for (int u = 0; u < kIrlsPer; ++u)
    if (tid + u * kIrlsThreads < E) part[tid + u * kIrlsThreads] = accv[u];
  // objective partial
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) objp += __shfl_xor(objp, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = objp;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < kIrlsThreads / 64; ++k) s += red[k];
    work[L.obj + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kIrlsThreads) irls_solve_kernel(int d, double* work, int last,
                                                                  int* status) {
  const IrlsLayout L(d);
  if (work[L.state + 2] != 0.0) return;
  __shared__ double G[kIrlsMaxD * kIrlsMaxD];
  __shared__ double rhs[kIrlsMaxD];
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int E = d * (d + 1) / 2 + d;
  for (int e = tid; e < E; e += kIrlsThreads) {
    double s = 0.0;
    for (int g = 0; g < kIrlsWgs; ++g) s += work[L.part + (size_t)g * ((size_t)d * d + d) + e];
    if (e < d * (d + 1) / 2) {
      int i = 0, rem = e;
      while (rem >= d - i) { rem -= d - i; ++i; }
      const int j = i + rem;
      G[i * d + j] = s;
      G[j * d + i] = s;
    } else {
      rhs[e - d * (d + 1) / 2] = s;
    }
  }
  if (tid == 0) bad = 0;
  __shared__ int stop;
  // objective at the x used by the Gram pass
  if (tid == 0) {
    stop = 0;
    double obj = 0.0;
    for (int g = 0; g < kIrlsWgs; ++g) obj += work[L.obj + g];
    const double prev = work[L.state + 1];
    double eta = work[L.state + 0];
    const double floor_eta = work[L.state + 3];
    work[L.state + 5] = obj;
    // smoothing floor: eta sum(w) <= 1e-10 of the current objective
    const double floor_now = 1e-10 * obj / work[L.state + 4];
    if (eta <= 0.0) {
      eta = obj / work[L.state + 4];  // first smoothing level: mean weighted residual
    } else {
      const bool at_floor = eta <= floor_eta * 1.0000001;
      if (at_floor && fabs(prev - obj) <= 1e-11 * obj) stop = 1;
      eta = fmax(floor_now, 0.5 * eta);
    }
    work[L.state + 3] = fmax(floor_now, 0.0);
    work[L.state + 1] = obj;
    work[L.state + 0] = eta;
  }
  __syncthreads();
  if (last || stop) {  // evaluation-only pass, or converged: keep x
    if (tid == 0 && stop) work[L.state + 2] = 1.0;
    return;
  }
  // Jacobi equilibration: G~ = S G S, rhs~ = S rhs with S = diag(1/sqrt(G_jj)),
  // so column scales of the weighted design do not enter the conditioning;
  // then Cholesky G~ = L L^T (in place, lower) and two triangular solves.
  __shared__ double sc[kIrlsMaxD];
  for (int k = tid; k < d; k += kIrlsThreads) {
    const double g = G[k * d + k];
    sc[k] = g > 0.0 ? 1.0 / sqrt(g) : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < d * d; e += kIrlsThreads) G[e] *= sc[e / d] * sc[e % d];
  for (int k = tid; k < d; k += kIrlsThreads) rhs[k] *= sc[k];
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    if (tid == 0) {
      const double gkk = G[k * d + k];
      if (!(gkk > 1e-15)) bad = 1;
      piv = sqrt(fmax(gkk, 1e-300));
      G[k * d + k] = piv;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < d; i += kIrlsThreads) G[i * d + k] /= piv;
    __syncthreads();
    for (int e = tid; e < (d - k - 1) * (d - k - 1); e += kIrlsThreads) {
      const int i = k + 1 + e / (d - k - 1), j = k + 1 + e % (d - k - 1);
      if (j <= i) G[i * d + j] -= G[i * d + k] * G[j * d + k];
    }
    __syncthreads();
  }
  // forward solve L y = rhs (column sweep), then L^T z = y; x = S z
  for (int k = 0; k < d; ++k) {
    if (tid == 0) rhs[k] /= G[k * d + k];
    __syncthreads();
    for (int i = k + 1 + tid; i < d; i += kIrlsThreads) rhs[i] -= G[i * d + k] * rhs[k];
    __syncthreads();
  }
  for (int k = d - 1; k >= 0; --k) {
    if (tid == 0) rhs[k] /= G[k * d + k];
    __syncthreads();
    for (int i = tid; i < k; i += kIrlsThreads) rhs[i] -= G[k * d + i] * rhs[k];
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) {
      *status = -4;
      work[L.state + 2] = 1.0;
    }
  } else {
    for (int i = tid; i < d; i += kIrlsThreads) work[L.x + i] = rhs[i] * sc[i];
  }
}

__global__ void __launch_bounds__(1024) irls_init_kernel(int d, const double* __restrict__ w,
                                                         const int64_t* S_dev, int64_t cap,
                                                         double* work) {
  const IrlsLayout L(d);
  __shared__ double red[16];
  const int64_t S = min(*S_dev, cap);
  double sw = 0.0;
  for (int64_t k = threadIdx.x; k < S; k += blockDim.x) sw += w[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sw += __shfl_xor(sw, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sw;
  if (threadIdx.x < d) work[L.x + threadIdx.x] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
    work[L.state + 0] = 0.0;
    work[L.state + 1] = 0.0;
    work[L.state + 2] = 0.0;
    work[L.state + 3] = 0.0;
    work[L.state + 4] = t > 0.0 ? t : 1.0;
    work[L.state + 5] = 0.0;
  }
}

__global__ void irls_out_kernel(int d, const double* work, double* x_out, double* obj_out) {
  const IrlsLayout L(d);
  if (threadIdx.x < d) x_out[threadIdx.x] = work[L.x + threadIdx.x];
  if (threadIdx.x == 0 && obj_out) *obj_out = work[L.state + 5];
}

hipError_t launch_irls(const void* At, const void* bt, const double* w, const int64_t* S_dev,
                       int64_t cap, int d, int64_t ldat, bool f64, int iters, double* work,
                       double* x_out, double* obj_out, int* status, hipStream_t st) {
  if (d > kIrlsMaxD || d < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(irls_init_kernel, dim3(1), dim3(1024), 0, st, d, w, S_dev, cap, work);
  for (int it = 0; it <= iters; ++it) {
    const int last = it == iters;
    if (f64)
      hipLaunchKernelGGL(irls_gram_kernel<double>, dim3(kIrlsWgs), dim3(kIrlsThreads), 0, st,
                         (const double*)At, (const double*)bt, w, S_dev, cap, d, ldat, work);
    else
      hipLaunchKernelGGL(irls_gram_kernel<float>, dim3(kIrlsWgs), dim3(kIrlsThreads), 0, st,
                         (const float*)At, (const float*)bt, w, S_dev, cap, d, ldat, work);
    hipLaunchKernelGGL(irls_solve_kernel, dim3(1), dim3(kIrlsThreads), 0, st, d, work, last,
                       status);
  }
  hipLaunchKernelGGL(irls_out_kernel, dim3(1), dim3(128), 0, st, d, work, x_out, obj_out);
  return hipGetLastError();
}

}  // namespace fctl1
