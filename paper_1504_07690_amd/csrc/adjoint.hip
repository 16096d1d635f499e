// Kernels of the adjoint of the estimate L = sum_i phibar_i phi~(t_i) with respect to
// the stored values of A (the hot path run backwards; not part of the paper).
//
//   Zbar_i = W Kbar_W,i + 2 Z_i Kbar_Z,i            (from K_W = sym(W^T Z), K_Z = Z^T Z)
//   Ybar_k = sum_i mu_k(t_i) Zbar_i                  (transposed sweep: the sweep kernels
//                                                    with the coefficient table transposed)
//   Lambda_k = Ybar_k + 2 A~ Lambda_{k+1} - Lambda_{k+2}   (the recurrence kernel)
//   abar_e += alpha c_k Lambda_k[r_e] . Y_{k-1}[c_e],  c_1 = 1, c_k = 2 (k >= 2)
#include "ssm_kernels.h"

namespace ssm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Zbar, in place over Z: one workgroup per (sweep point, run of rows).  The
// (2 N_v) x N_v stack [Kbar_W; 2 Kbar_Z] sits in LDS as FP64; each wave takes 16
// rows at a time and multiplies [W | Z] (16 x 2 N_v) by it on
// v_mfma_f64_16x16x4_f64, T = N_v/16 output blocks per wave.  A wave reads only
// the rows it writes, and writes them after its last read of them.
// ---------------------------------------------------------------------------
constexpr int ZB_ROWS_PER_BLOCK = 1024;

template <int T, typename In>
__global__ void __launch_bounds__(256) zbar_kernel(int64_t n, int nv, const In* __restrict__ w, In* __restrict__ z,
                                                   const double* __restrict__ kw_bar,
                                                   const double* __restrict__ kz_bar) {
  extern __shared__ double kb[];  // [2 nv][16 T]
  constexpr int NP = 16 * T;
  const int i = blockIdx.y;
  const int64_t nn = (int64_t)nv * nv;
  const double* kwb = kw_bar + i * nn;
  const double* kzb = kz_bar + i * nn;
  for (int idx = threadIdx.x; idx < 2 * nv * NP; idx += blockDim.x) {
    const int r = idx / NP, c = idx % NP;
    double v = 0.0;
    if (c < nv) v = (r < nv) ? kwb[(int64_t)r * nv + c] : 2.0 * kzb[(int64_t)(r - nv) * nv + c];
    kb[idx] = v;
  }
  __syncthreads();
  In* zi = z + (int64_t)i * n * nv;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r_begin = (int64_t)blockIdx.x * ZB_ROWS_PER_BLOCK;
  const int64_t r_end = (r_begin + ZB_ROWS_PER_BLOCK < n) ? r_begin + ZB_ROWS_PER_BLOCK : n;
  for (int64_t r0 = r_begin + 16 * wave; r0 < r_end; r0 += 64) {
    const int64_t row = r0 + (lane & 15);
    const bool rok = row < r_end;
    f64x4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // contraction over q < 2 nv (<= 2 NP), four at a time: A[m = lane%16][k = lane/16];
    // the whole 16 x 2 nv slab is loaded before the MFMAs that use it
    constexpr int KQ = 2 * NP / 4;
    In av[KQ];
#pragma unroll
    for (int s = 0; s < KQ; ++s) {
      const int q = 4 * s + (lane >> 4);
      In v = (In)0;
      if (rok && q < 2 * nv) v = (q < nv) ? w[row * nv + q] : zi[row * nv + (q - nv)];
      av[s] = v;
    }
#pragma unroll
    for (int s = 0; s < KQ; ++s) {
      const int q = 4 * s + (lane >> 4);
      const double a = (double)av[s];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const double bv = (q < 2 * nv) ? kb[q * NP + 16 * t + (lane & 15)] : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
      }
    }
    // result register r of lane l holds D[l/16 + 4r][l%16]; every read of these
    // rows by this wave is complete (the MFMA results depend on all of them)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int col = 16 * t + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = r0 + (lane >> 4) + 4 * r;
        if (orow < r_end && col < nv) zi[orow * nv + col] = (In)acc[t][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// SDDMM on the pattern of A: abar[e] += coef * sum_j lam[r_e][j] y[c_e][j], one
// thread per stored entry, FP64 sums.
// ---------------------------------------------------------------------------
template <typename In>
__global__ void __launch_bounds__(256) sddmm_kernel(int64_t nnz, int nv, const int32_t* __restrict__ row_of,
                                                    const int32_t* __restrict__ col_idx, const In* __restrict__ lam,
                                                    const In* __restrict__ y, double coef, double* __restrict__ abar) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const In* lr = lam + (int64_t)row_of[e] * nv;
  const In* yc = y + (int64_t)col_idx[e] * nv;
  double acc = 0.0;
  for (int j = 0; j < nv; ++j) acc += (double)lr[j] * (double)yc[j];
  abar[e] += coef * acc;
}

__global__ void __launch_bounds__(256) row_of_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ row_of) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int p = row_ptr[r]; p < row_ptr[r + 1]; ++p) row_of[p] = (int32_t)r;
}

// ct[i*ldct + k] = c[k*ldc + i] (FP64 and FP32 copies), zero padded to ldct
__global__ void __launch_bounds__(256) transpose_coefficients_kernel(const double* __restrict__ c, int64_t ldc, int nt,
                                                                     int m1, double* __restrict__ ct64,
                                                                     float* __restrict__ ct32, int64_t ldct) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nt * ldct) return;
  const int i = (int)(gid / ldct);
  const int k = (int)(gid - (int64_t)i * ldct);
  const double v = k < m1 ? c[(int64_t)k * ldc + i] : 0.0;
  if (ct64) ct64[gid] = v;
  if (ct32) ct32[gid] = (float)v;
}

template <int T>
hipError_t launch_zbar_t(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kwb,
                         const double* kzb, hipStream_t stream) {
  const size_t lds = (size_t)2 * nv * 16 * T * sizeof(double);
  dim3 grid((unsigned)((n + ZB_ROWS_PER_BLOCK - 1) / ZB_ROWS_PER_BLOCK), ntb);
  hipError_t err;
  if (is_f32) {
    err = hipFuncSetAttribute((const void*)zbar_kernel<T, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((zbar_kernel<T, float>), grid, dim3(256), lds, stream, n, nv, (const float*)w, (float*)z, kwb,
                       kzb);
  } else {
    err = hipFuncSetAttribute((const void*)zbar_kernel<T, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((zbar_kernel<T, double>), grid, dim3(256), lds, stream, n, nv, (const double*)w, (double*)z,
                       kwb, kzb);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zbar(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kw_bar,
                       const double* kz_bar, hipStream_t stream) {
  switch ((nv + 15) / 16) {
    case 1: return launch_zbar_t<1>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 2: return launch_zbar_t<2>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 3: return launch_zbar_t<3>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 4: return launch_zbar_t<4>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 5: return launch_zbar_t<5>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 6: return launch_zbar_t<6>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sddmm(int is_f32, int64_t nnz, int nv, const int32_t* row_of, const int32_t* col_idx,
                        const void* lam, const void* y, double coef, double* abar, hipStream_t stream) {
  const unsigned blocks = (unsigned)((nnz + 255) / 256);
  if (is_f32)
    hipLaunchKernelGGL(sddmm_kernel<float>, dim3(blocks), dim3(256), 0, stream, nnz, nv, row_of, col_idx,
                       (const float*)lam, (const float*)y, coef, abar);
  else
    hipLaunchKernelGGL(sddmm_kernel<double>, dim3(blocks), dim3(256), 0, stream, nnz, nv, row_of, col_idx,
                       (const double*)lam, (const double*)y, coef, abar);
  return hipGetLastError();
}

hipError_t launch_row_of(int64_t n, const int32_t* row_ptr, int32_t* row_of, hipStream_t stream) {
  hipLaunchKernelGGL(row_of_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, row_ptr, row_of);
  return hipGetLastError();
}

hipError_t launch_transpose_coefficients(const double* c, int64_t ldc, int nt, int m1, double* ct64, float* ct32,
                                         int64_t ldct, hipStream_t stream) {
  const int64_t total = (int64_t)nt * ldct;
  hipLaunchKernelGGL(transpose_coefficients_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, c,
                     ldc, nt, m1, ct64, ct32, ldct);
  return hipGetLastError();
}


}  // namespace ssm
