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
