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
