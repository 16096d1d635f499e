// Sum of squares of a block, in FP64, in two fixed-order stages (bitwise
// reproducible).  Used for the bound check ||T_M(A~) W||_F <= ||W||_F, which
// holds because |T_k| <= 1 on [-1, 1] when spec(A~) lies in [-1, 1].
#include "ssm_kernels.h"

namespace ssm {
namespace {

constexpr int kPartials = 1024;

template <typename T>
__global__ void __launch_bounds__(256) sumsq_stage1(const T* __restrict__ x, int64_t count, double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) sumsq_stage2(const double* __restrict__ partial, int np, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

int reduce_partials() { return kPartials; }

hipError_t launch_sumsq(const void* x, int64_t count, int is_f32, double* partial, double* out,
                        hipStream_t stream) {
  if (is_f32)
    hipLaunchKernelGGL(sumsq_stage1<float>, dim3(kPartials), dim3(256), 0, stream, (const float*)x, count,
                       partial);
  else
    hipLaunchKernelGGL(sumsq_stage1<double>, dim3(kPartials), dim3(256), 0, stream, (const double*)x, count,
                       partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(sumsq_stage2, dim3(1), dim3(256), 0, stream, partial, kPartials, out);
  return hipGetLastError();
}

}  // namespace ssm
