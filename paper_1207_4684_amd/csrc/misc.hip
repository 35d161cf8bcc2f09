// Data preparation and verification kernels: the BF16 copy streamed by the
// precision form of the sampling pass, and the full l1 objective
// ||A x - b||_1 used to check the (1 + eps) guarantee of the regression
// theorem (not part of the method's own path).
#include "fct_device.h"
#include "fct_kernels.h"

namespace fctl1 {

// Grid-stride: the dispatch's work-item count is a 32-bit quantity, so the
// grid is capped and each thread converts several elements.
__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t count, uint16_t* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = __float_as_uint(x[i]);
    y[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
}

hipError_t launch_to_bf16(const float* x, int64_t count, uint16_t* y, hipStream_t st) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, count, y);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) l1_objective_kernel(const T* __restrict__ A,
                                                           const T* __restrict__ b, int64_t lda,
                                                           int64_t n, int d,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ parts) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r = -(double)b[i];
    for (int c = 0; c < d; ++c) r = fma((double)A[i + (int64_t)c * lda], x[c], r);
    s += fabs(r);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_l1_objective(const void* A, const void* b, int64_t lda, int64_t n, int d,
                               const double* x, bool f64, double* parts, int nparts, double* out,
                               hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(l1_objective_kernel<double>, dim3(nparts), dim3(256), 0, st,
                       (const double*)A, (const double*)b, lda, n, d, x, parts);
  else
    hipLaunchKernelGGL(l1_objective_kernel<float>, dim3(nparts), dim3(256), 0, st,
                       (const float*)A, (const float*)b, lda, n, d, x, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_fixed(parts, nparts, out, st);
}

}  // namespace fctl1

namespace fctl1 {

// The residual form of X for a low-precision sampling pass.  With
// R = [R_AA r_Ab; 0 r_bb] the R factor of the sketch of X = [A, -b], the
// sketched least-squares solution x0 solves R_AA x0 = -r_Ab, and with
// T = [I x0; 0 1]: X T = [A, A x0 - b] = [A, -r0], r0 = b - A x0, and
// (X T)(R T)^-1 = X R^-1, so the row-norm estimates are unchanged while the
// last column, rounded to BF16, carries the residual instead of b.
// One thread: back substitution (d <= 64) and R T (column d replaced by
// R_AA x0 + r_Ab, formed explicitly).
__global__ void lowp_basis_kernel(const double* __restrict__ R, int d, double* __restrict__ x0,
                                  double* __restrict__ R_res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int q = d + 1;
  for (int i = d - 1; i >= 0; --i) {
    double t = -R[i + (int64_t)d * q];
    for (int j = i + 1; j < d; ++j) t -= R[i + (int64_t)j * q] * x0[j];
    x0[i] = t / R[i + (int64_t)i * q];
  }
  for (int k = 0; k < q * q; ++k) R_res[k] = R[k];
  for (int i = 0; i < d; ++i) {
    double t = R[i + (int64_t)d * q];
    for (int j = i; j < d; ++j) t = fma(R[i + (int64_t)j * q], x0[j], t);
    R_res[i + (int64_t)d * q] = t;
  }
}

// r0_i = b_i - A_i x0 in FP64, stored as BF16 (rounded to FP32, then to the
// nearest BF16, ties to even, as the BF16 copy of A is).
template <typename T>
__global__ void __launch_bounds__(256) residual_bf16_kernel(const T* __restrict__ A,
                                                            const T* __restrict__ b, int64_t lda,
                                                            int64_t n, int d,
                                                            const double* __restrict__ x0,
                                                            uint16_t* __restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double t = (double)b[i];
    for (int c = 0; c < d; ++c) t = fma(-(double)A[i + (int64_t)c * lda], x0[c], t);
    const uint32_t u = __float_as_uint((float)t);
    r[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  }
}

hipError_t launch_lowp_residual(const void* A, const void* b, int64_t lda, int64_t n, int d,
                                bool f64, const double* R, double* x0, double* R_res, uint16_t* r,
                                hipStream_t st) {
  hipLaunchKernelGGL(lowp_basis_kernel, dim3(1), dim3(64), 0, st, R, d, x0, R_res);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (f64)
    hipLaunchKernelGGL(residual_bf16_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const double*)A, (const double*)b, lda, n, d, x0, r);
  else
    hipLaunchKernelGGL(residual_bf16_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const float*)A, (const float*)b, lda, n, d, x0, r);
  return hipGetLastError();
}

}  // namespace fctl1

namespace fctl1 {

// sum_i |(A W)_ij - B_ij| for the k columns of W (d x k, column-major,
// FP64; B optional, n x k with leading dimension ldb), in FP64.  The grid's
// y index takes 8 consecutive columns; a thread takes rows in a grid stride
// and keeps its 8 sums in registers; a workgroup's sums go to
// parts[blockIdx.x][j] after a fixed-order reduction.
template <typename T>
__global__ void __launch_bounds__(256) l1_objectives_kernel(const T* __restrict__ A,
                                                            const T* __restrict__ B, int64_t lda,
                                                            int64_t ldb, int64_t n, int d, int k,
                                                            const double* __restrict__ W,
                                                            double* __restrict__ parts) {
  __shared__ double red[4][8];
  const int j0 = blockIdx.y * 8;
  double s[8];
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) s[jj] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
      r[jj] = (B && j0 + jj < k) ? -(double)B[i + (int64_t)(j0 + jj) * ldb] : 0.0;
    for (int c = 0; c < d; ++c) {
      const double a = (double)A[i + (int64_t)c * lda];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (j0 + jj < k) r[jj] = fma(a, W[c + (int64_t)(j0 + jj) * d], r[jj]);
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) s[jj] += fabs(r[jj]);
  }
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const double v = wave_sum_dpp(s[jj]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][jj] = v;
  }
  __syncthreads();
  if (threadIdx.x < 8 && j0 + (int)threadIdx.x < k)
    parts[(int64_t)blockIdx.x * k + j0 + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// out[j] = sum over the workgroups of parts[.][j], in workgroup order
__global__ void objectives_sum_kernel(const double* __restrict__ parts, int nparts, int k,
                                      double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += parts[(int64_t)p * k + j];
  out[j] = s;
}

hipError_t launch_l1_objectives(const void* A, const void* B, int64_t lda, int64_t ldb, int64_t n,
                                int d, int k, const double* W, bool f64, double* parts, int nparts,
                                double* out, hipStream_t st) {
  const dim3 grid((unsigned)nparts, (unsigned)((k + 7) / 8));
  if (f64)
    hipLaunchKernelGGL(l1_objectives_kernel<double>, grid, dim3(256), 0, st, (const double*)A,
                       (const double*)B, lda, ldb, n, d, k, W, parts);
  else
    hipLaunchKernelGGL(l1_objectives_kernel<float>, grid, dim3(256), 0, st, (const float*)A,
                       (const float*)B, lda, ldb, n, d, k, W, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(objectives_sum_kernel, dim3((unsigned)((k + 63) / 64)), dim3(64), 0, st, parts,
                     nparts, k, out);
  return hipGetLastError();
}

// The d designs of the constrained regressions of subspace approximation:
// for column j, the coreset's other d - 1 columns (in order) into
// Aj[j][.] and column j into bj[j][.] (each cap rows, leading dimension cap).
template <typename T>
__global__ void __launch_bounds__(256) drop_column_kernel(const T* __restrict__ At, int64_t cap, int d,
                                                          const int64_t* __restrict__ S,
                                                          T* __restrict__ Aj, T* __restrict__ bj) {
  const int j = blockIdx.y;
  const int64_t cnt = min(*S, cap);
  T* dst = Aj + (int64_t)j * cap * (d - 1);
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < cnt;
       r += (int64_t)gridDim.x * blockDim.x) {
    for (int c = 0, o = 0; c < d; ++c) {
      const T v = At[r + (int64_t)c * cap];
      if (c == j) bj[(int64_t)j * cap + r] = v;
      else dst[r + (int64_t)(o++) * cap] = v;
    }
  }
}

hipError_t launch_drop_column(const void* At, int64_t cap, int d, const int64_t* S, void* Aj,
                              void* bj, bool f64, hipStream_t st) {
  int64_t gx = (cap + 255) / 256;
  if (gx > 1024) gx = 1024;
  const dim3 grid((unsigned)gx, (unsigned)d);
  if (f64)
    hipLaunchKernelGGL(drop_column_kernel<double>, grid, dim3(256), 0, st, (const double*)At, cap,
                       d, S, (double*)Aj, (double*)bj);
  else
    hipLaunchKernelGGL(drop_column_kernel<float>, grid, dim3(256), 0, st, (const float*)At, cap,
                       d, S, (float*)Aj, (float*)bj);
  return hipGetLastError();
}

}  // namespace fctl1
