// Algorithm 1 (Delta-Gauss-Chebyshev coefficients) for all sweep points at once.
//
// mu_l(t) = (2 - delta_l0) / (2 N_theta) * Re sum_{j<2N_theta} exp(-i 2 pi j l / 2N_theta) g_j,
// g_j = g_sigma(t - x(cos theta_j)), theta_j = j pi / N_theta   (Eq. mucoef2 discretised).
// Because cos(theta_{2N_theta - j}) = cos(theta_j), g is even in j and the DFT is a
// cosine sum over j = 0..N_theta (a DCT-I):
//   Re g^_l = g_0 + (-1)^l g_{N_theta} + 2 sum_{0<j<N_theta} g_j cos(pi j l / N_theta).
// One workgroup per sweep point: g_j and the table cos(pi m / N_theta), m = 0..N_theta,
// sit in LDS; the index j*l is reduced modulo 2 N_theta exactly, in integers.
#include "ssm_kernels.h"

namespace ssm {
namespace {

__global__ void __launch_bounds__(256) dgc_coefficients_kernel(double c0, double hw, double sigma,
                                                               double inv_norm, const double* __restrict__ t,
                                                               int nt, int degree, int n_theta,
                                                               double* __restrict__ c,
                                                               float* __restrict__ c32, int64_t ldc) {
  extern __shared__ double lds[];
  double* g = lds;                 // n_theta + 1
  double* cs = lds + n_theta + 1;  // n_theta + 1
  const int i = blockIdx.x;
  const double ti = t[i];
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  for (int j = threadIdx.x; j <= n_theta; j += blockDim.x) {
    const double ct = cospi((double)j / (double)n_theta);
    cs[j] = ct;
    const double s = ti - (c0 + hw * ct);
    g[j] = inv_norm * exp(-s * s * inv2s2);
  }
  __syncthreads();
  const int two = 2 * n_theta;
  for (int l = threadIdx.x; l <= degree; l += blockDim.x) {
    double acc = 0.0;
    int m = 0;
    for (int j = 1; j < n_theta; ++j) {
      m += l;
      if (m >= two) m -= two;  // l < 2 N_theta, so one subtraction keeps m = (j l) mod 2N_theta
      const int idx = (m <= n_theta) ? m : two - m;
      acc += g[j] * cs[idx];
    }
    const double re = g[0] + ((l & 1) ? -g[n_theta] : g[n_theta]) + 2.0 * acc;
    const double mu = re / (double)two * (l == 0 ? 1.0 : 2.0);
    c[(int64_t)l * ldc + i] = mu;
    if (c32) c32[(int64_t)l * ldc + i] = (float)mu;
  }
}

// Proposition 1: nu_l(t_i), l = 0..2h, of the square of sum_{k<=h} mu_k(t_i) T_k.  With
// T_p T_q = (T_{p+q} + T_{|p-q|}) / 2 over ordered pairs (p, q),
//   nu_l = 1/2 sum_{p+q=l} mu_p mu_q + 1/2 sum_{|p-q|=l} mu_p mu_q,
// the second sum being sum_p mu_p^2 for l = 0 and 2 sum_p mu_p mu_{p+l} otherwise: the
// exact coefficients (the quadrature the proposition names gives the same numbers for
// N_theta > 2h).  One lane per (l, column); columns nt..ldn-1 are written as 0.
__global__ void __launch_bounds__(256) square_coefficients_kernel(const double* __restrict__ mu, int64_t ldc,
                                                                  int nt, int h, int64_t ldn,
                                                                  double* __restrict__ nu) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m1 = 2 * h + 1;
  if (idx >= (int64_t)m1 * ldn) return;
  const int l = (int)(idx / ldn);
  const int i = (int)(idx - (int64_t)l * ldn);
  if (i >= nt) {
    nu[idx] = 0.0;
    return;
  }
  double conv = 0.0;  // p + q = l
  const int p_lo = l > h ? l - h : 0;
  const int p_hi = l < h ? l : h;
  for (int p = p_lo; p <= p_hi; ++p) conv += mu[(int64_t)p * ldc + i] * mu[(int64_t)(l - p) * ldc + i];
  double diff = 0.0;  // |p - q| = l
  for (int p = 0; p + l <= h; ++p) diff += mu[(int64_t)p * ldc + i] * mu[(int64_t)(p + l) * ldc + i];
  if (l > 0) diff *= 2.0;
  nu[idx] = 0.5 * (conv + diff);
}

}  // namespace

hipError_t launch_square_coefficients(const double* mu, int64_t ldc, int nt, int h, double* nu, int64_t ldn,
                                      hipStream_t stream) {
  const int64_t total = (int64_t)(2 * h + 1) * ldn;
  hipLaunchKernelGGL(square_coefficients_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, mu, ldc,
                     nt, h, ldn, nu);
  return hipGetLastError();
}

namespace {

// mun[i] = sqrt(sum_l c[l][i]^2): 64 points per workgroup, four waves splitting the degrees
// in interleaved quarters, summed in a fixed order (deterministic)
__global__ void __launch_bounds__(256) coefficient_norms_kernel(const double* __restrict__ c, int64_t ldc, int nt,
                                                                int m1, double* __restrict__ mun) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (i < nt)
    for (int l = q; l < m1; l += 4) {
      const double v = c[(int64_t)l * ldc + i];
      acc += v * v;
    }
  part[q][lane] = acc;
  __syncthreads();
  if (q == 0 && i < nt) mun[i] = sqrt(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

// kmax[l] = max_i |c[l][i]|: one workgroup per degree
__global__ void __launch_bounds__(256) coefficient_row_max_kernel(const double* __restrict__ c, int64_t ldc, int nt,
                                                                  double* __restrict__ kmax) {
  __shared__ double red[256];
  const double* row = c + (int64_t)blockIdx.x * ldc;
  double m = 0.0;
  for (int i = threadIdx.x; i < nt; i += 256) m = fmax(m, fabs(row[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) kmax[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) rounding_floor_kernel(const double* __restrict__ mun, int nt, double eta,
                                                             const double* __restrict__ w_sumsq, double inv_sqrt_e,
                                                             double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nt) out[i] = eta * mun[i] * (w_sumsq[0] * inv_sqrt_e);
}

}  // namespace

hipError_t launch_coefficient_norms(const double* c, int64_t ldc, int nt, int m1, double* mun, hipStream_t stream) {
  hipLaunchKernelGGL(coefficient_norms_kernel, dim3((unsigned)((nt + 63) / 64)), dim3(256), 0, stream, c, ldc, nt, m1,
                     mun);
  return hipGetLastError();
}

hipError_t launch_coefficient_row_max(const double* c, int64_t ldc, int nt, int m1, double* kmax,
                                      hipStream_t stream) {
  hipLaunchKernelGGL(coefficient_row_max_kernel, dim3((unsigned)m1), dim3(256), 0, stream, c, ldc, nt, kmax);
  return hipGetLastError();
}

hipError_t launch_rounding_floor(const double* mun, int nt, double eta, const double* w_sumsq, double inv_sqrt_e,
                                 double* floor_out, hipStream_t stream) {
  hipLaunchKernelGGL(rounding_floor_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, stream, mun, nt, eta,
                     w_sumsq, inv_sqrt_e, floor_out);
  return hipGetLastError();
}

size_t coefficient_lds_bytes(int n_theta) { return 2 * (size_t)(n_theta + 1) * sizeof(double); }

hipError_t launch_coefficients(double c0, double hw, double sigma, double inv_norm, const double* t, int nt,
                               int degree, int n_theta, double* c, float* c32, int64_t ldc,
                               hipStream_t stream) {
  const size_t lds = coefficient_lds_bytes(n_theta);
  hipError_t err = hipFuncSetAttribute((const void*)dgc_coefficients_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(dgc_coefficients_kernel, dim3(nt), dim3(256), lds, stream, c0, hw, sigma, inv_norm, t,
                     nt, degree, n_theta, c, c32, ldc);
  return hipGetLastError();
}

}  // namespace ssm
