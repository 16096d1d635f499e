// RESS-DGC (Algorithm 7, Theorem 4): the moments X_l = V^T T_l(A~) V of the block
// V = [W W~] (N x N_v', N_v' = N_v + N~_v) for l = 0..M, and their split into the
// per-point matrices of Algorithms 4 and 6.
//
// The recurrence runs only to Y_{M/2+1}: the pair Gram kernel gives, for s = 0..M/2,
//   pw[s] = (Y_{s+1}^T Y_s + Y_s^T Y_{s+1}) / 2,   pz[s] = Y_s^T Y_s,
// and for symmetric A~, T_s^2 = (T_{2s} + T_0)/2 and T_{s+1} T_s = (T_{2s+1} + T_1)/2 give
//   X_0 = pz[0],  X_1 = pw[0],  X_{2s} = 2 pz[s] - X_0,  X_{2s+1} = 2 pw[s] - X_1.
// The per-point sums K_mu(t_i) = sum_{l<=M/2} mu_l(t_i) X_l and K_nu(t_i) = sum_{l<=M}
// nu_l(t_i) X_l are the FP64 sweep GEMM over X (blocks of N_v'^2 entries); this file
// then cuts K_W, K_Z (upper-left N_v x N_v), K_C (lower-left N~_v x N_v) and Tr K_W~
// (trace of the lower-right N~_v x N~_v block) out of them.
#include "ssm_kernels.h"

namespace ssm {
namespace {

__global__ void __launch_bounds__(256) ress_moments_kernel(int64_t nn, int m1, const double* __restrict__ pw,
                                                           const double* __restrict__ pz, double* __restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m1 * nn) return;
  const int l = (int)(idx / nn);
  const int64_t q = idx - (int64_t)l * nn;
  const int s = l >> 1;
  const double* src = (l & 1) ? pw : pz;
  double v = src[(int64_t)s * nn + q];
  if (s > 0) v = 2.0 * v - src[q];
  x[idx] = v;
}

// One workgroup per point.
__global__ void __launch_bounds__(256) ress_extract_kernel(int nv, int nvh, const double* __restrict__ kmu,
                                                           const double* __restrict__ knu, double* __restrict__ kw,
                                                           double* __restrict__ kz, double* __restrict__ kc,
                                                           double* __restrict__ trw) {
  const int i = blockIdx.x;
  const int nvp = nv + nvh;
  const int64_t nnp = (int64_t)nvp * nvp;
  const double* mu_i = kmu + i * nnp;
  const double* nu_i = knu + i * nnp;
  for (int idx = threadIdx.x; idx < nv * nv; idx += blockDim.x) {
    const int r = idx / nv, c = idx - r * nv;
    kw[(int64_t)i * nv * nv + idx] = mu_i[(int64_t)r * nvp + c];
    kz[(int64_t)i * nv * nv + idx] = nu_i[(int64_t)r * nvp + c];
  }
  if (nvh == 0) return;
  for (int idx = threadIdx.x; idx < nvh * nv; idx += blockDim.x) {
    const int r = idx / nv, c = idx - r * nv;
    kc[(int64_t)i * nvh * nv + idx] = mu_i[(int64_t)(nv + r) * nvp + c];
  }
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int j = nv; j < nvp; ++j) tr += mu_i[(int64_t)j * nvp + j];
    trw[i] = tr;
  }
}

// Rounding floor of the truncation: K_W(t_i) = sum_{l<=h} mu_l(t_i) X_l[:nv, :nv] rounds at
// about u sum_l |mu_l(t_i)| max|X_l[:nv, :nv]|, so Algorithm 4 also drops eigenvalues below
// eta times that sum.  One workgroup per l for the maxima (fixed order), then one lane
// per point.
__global__ void __launch_bounds__(256) ress_xmax_kernel(int nv, int nvp, const double* __restrict__ x,
                                                        double* __restrict__ xmax) {
  __shared__ double red[256];
  const double* xl = x + (int64_t)blockIdx.x * nvp * nvp;
  double m = 0.0;
  for (int idx = threadIdx.x; idx < nv * nv; idx += 256) {
    const int r = idx / nv, c = idx - r * nv;
    m = fmax(m, fabs(xl[(int64_t)r * nvp + c]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) xmax[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) ress_floor_kernel(const double* __restrict__ mu, int64_t ldc, int nt, int h,
                                                         const double* __restrict__ xmax, double eta,
                                                         double* __restrict__ floor_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  double acc = 0.0;
  for (int l = 0; l <= h; ++l) acc += fabs(mu[(int64_t)l * ldc + i]) * xmax[l];
  floor_out[i] = eta * acc;
}

}  // namespace

hipError_t launch_ress_floor(int nv, int nvp, int h, const double* x, const double* mu, int64_t ldc, int nt,
                             double eta, double* xmax, double* floor_out, hipStream_t stream) {
  hipLaunchKernelGGL(ress_xmax_kernel, dim3(h + 1), dim3(256), 0, stream, nv, nvp, x, xmax);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(ress_floor_kernel, dim3((nt + 255) / 256), dim3(256), 0, stream, mu, ldc, nt, h, xmax, eta,
                     floor_out);
  return hipGetLastError();
}

hipError_t launch_ress_moments(int nvp, int m1, const double* pw, const double* pz, double* x, hipStream_t stream) {
  const int64_t nn = (int64_t)nvp * nvp;
  const int64_t total = (int64_t)m1 * nn;
  hipLaunchKernelGGL(ress_moments_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, nn, m1, pw, pz,
                     x);
  return hipGetLastError();
}

hipError_t launch_ress_extract(int nt, int nv, int nvh, const double* kmu, const double* knu, double* kw, double* kz,
                               double* kc, double* trw, hipStream_t stream) {
  hipLaunchKernelGGL(ress_extract_kernel, dim3(nt), dim3(256), 0, stream, nv, nvh, kmu, knu, kw, kz, kc, trw);
  return hipGetLastError();
}

}  // namespace ssm
