// The Gaussian block W of Section 2 (entries i.i.d. N(0,1)), drawn on the device.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 and forms
// (hi(w2 M1) ^ w1 ^ k0, lo(w2 M1), hi(w0 M0) ^ w3 ^ k1, lo(w0 M0)); the key is
// advanced by 0x9E3779B9 and 0xBB67AE85 between rounds.
// Element (r, 4g + m) is normal m of counter (g, 0, r mod 2^32, r div 2^32) under
// key (seed mod 2^32, seed div 2^32); Box-Muller turns (x0, x1) into normals 0, 1
// and (x2, x3) into normals 2, 3 with u = (x_even + 1) 2^-32, v = x_odd 2^-32.
#include "ssm_kernels.h"

namespace ssm {
namespace {

__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * x0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t n0 = hi1 ^ x1 ^ k0;
    const uint32_t n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double u = ((double)a + 1.0) * 0x1p-32;
  const double v = (double)b * 0x1p-32;
  const double rad = sqrt(-2.0 * log(u));
  double s, c;
  sincospi(2.0 * v, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

template <typename T>
__global__ void __launch_bounds__(256) gaussian_block_kernel(uint64_t seed, int64_t n, int nv, T* __restrict__ w) {
  const int ng = (nv + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * ng) return;
  const int64_t r = gid / ng;
  const int g = (int)(gid - r * ng);
  uint32_t x0 = (uint32_t)g, x1 = 0u, x2 = (uint32_t)(r & 0xFFFFFFFF), x3 = (uint32_t)(r >> 32);
  philox4x32_10(x0, x1, x2, x3, (uint32_t)(seed & 0xFFFFFFFF), (uint32_t)(seed >> 32));
  double z[4];
  box_muller(x0, x1, z[0], z[1]);
  box_muller(x2, x3, z[2], z[3]);
  T* row = w + r * nv;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int j = 4 * g + m;
    if (j < nv) row[j] = (T)z[m];
  }
}

}  // namespace

hipError_t launch_gaussian_block(uint64_t seed, int64_t n, int nv, int dtype, void* w, hipStream_t stream) {
  const int64_t threads = n * ((nv + 3) / 4);
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(gaussian_block_kernel<double>, dim3(blocks), dim3(256), 0, stream, seed, n, nv,
                       (double*)w);
  else
    hipLaunchKernelGGL(gaussian_block_kernel<float>, dim3(blocks), dim3(256), 0, stream, seed, n, nv,
                       (float*)w);
  return hipGetLastError();
}

}  // namespace ssm
