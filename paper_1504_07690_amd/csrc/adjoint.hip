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

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Zbar, in place over Z: one workgroup per (sweep point, run of rows).  The
// stack [Kbar_W; 2 Kbar_Z] sits in LDS as FP64 (two 16T x 16T halves); each wave takes 16
// rows at a time and multiplies [W | Z] (16 x 2 N_v) by it on
// v_mfma_f64_16x16x4_f64, T = N_v/16 output blocks per wave.  A wave reads only
// the rows it writes, and writes them after its last read of them.
// ---------------------------------------------------------------------------
constexpr int ZB_ROWS_PER_BLOCK = 4096;

template <int T, typename In>
__global__ void __launch_bounds__(256) zbar_kernel(int64_t n, int nv, const In* __restrict__ w, In* __restrict__ z,
                                                   const double* __restrict__ kw_bar,
                                                   const double* __restrict__ kz_bar) {
  // [Kbar_W; 2 Kbar_Z] as two NP x NP halves (rows and columns past N_v zero), so that
  // the contraction index q < 2 NP needs no bounds test
  extern __shared__ double kb[];
  constexpr int NP = 16 * T;
  constexpr int KQ = 2 * NP / 4;  // contraction steps of four
  const int i = blockIdx.y;
  const int64_t nn = (int64_t)nv * nv;
  const double* kwb = kw_bar + i * nn;
  const double* kzb = kz_bar + i * nn;
  // stack fill: eight loads in flight per thread before their LDS stores
  constexpr int total = 2 * NP * NP;
  for (int base = threadIdx.x; base < total; base += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + 256 * u;
      const int r = idx / NP, c = idx % NP;
      const int hr = r < NP ? r : r - NP;  // row inside its half
      double x = 0.0;
      if (idx < total && c < nv && hr < nv) x = (r < NP) ? kwb[(int64_t)hr * nv + c] : 2.0 * kzb[(int64_t)hr * nv + c];
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (base + 256 * u < total) kb[base + 256 * u] = v[u];
  }
  __syncthreads();
  In* zi = z + (int64_t)i * n * nv;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r_begin = (int64_t)blockIdx.x * ZB_ROWS_PER_BLOCK;
  const int64_t r_end = (r_begin + ZB_ROWS_PER_BLOCK < n) ? r_begin + ZB_ROWS_PER_BLOCK : n;
  // the 16 x 2 NP slab of [W | Z] for rows r0 .. r0+15: A[m = lane%16][k = 4 s + lane/16];
  // indices are clamped into the arrays (rows past the range, columns past N_v), and the
  // values they bring meet zero stack rows or feed rows that are not stored
  auto load_slab = [&](int64_t r0, In (&av)[KQ]) {
    int64_t row = r0 + (lane & 15);
    row = row < r_end ? row : r_end - 1;
    const In* wr = w + row * nv;
    const In* zr = zi + row * nv;
#pragma unroll
    for (int s = 0; s < KQ; ++s) {
      const int q = 4 * s + (lane >> 4);
      const int c = (q < NP ? q : q - NP);
      const int cc = c < nv ? c : nv - 1;
      av[s] = (q < NP) ? wr[cc] : zr[cc];
    }
  };
  In cur[KQ], nxt[KQ];
  int64_t r0 = r_begin + 16 * wave;
  if (r0 < r_end) load_slab(r0, cur);
  for (; r0 < r_end; r0 += 64) {
    // the next slab's loads are in flight behind this slab's MFMAs
    if (r0 + 64 < r_end) load_slab(r0 + 64, nxt);
    f64x4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    // the stack operands of step s + 1 are read from LDS behind the MFMAs of step s
    const double* kbl = kb + (lane >> 4) * NP + (lane & 15);
    double bcur[T], bnxt[T];
#pragma unroll
    for (int t = 0; t < T; ++t) bcur[t] = kbl[16 * t];
#pragma unroll
    for (int s = 0; s < KQ; ++s) {
      if (s + 1 < KQ) {
#pragma unroll
        for (int t = 0; t < T; ++t) bnxt[t] = kbl[4 * (s + 1) * NP + 16 * t];
      }
      const double a = (double)cur[s];
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bcur[t], acc[t], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < T; ++t) bcur[t] = bnxt[t];
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
#pragma unroll
    for (int s = 0; s < KQ; ++s) cur[s] = nxt[s];
  }
}

// N_v above 96: the stack does not fit in LDS; the same MFMA walk reads [Kbar_W;
// 2 Kbar_Z] through the cache (one point's stack is shared by all its row blocks),
// and the 16 x 2 N_v slab is loaded eight k-steps at a time.
template <int T, typename In>
__global__ void __launch_bounds__(256) zbar_big_kernel(int64_t n, int nv, const In* __restrict__ w,
                                                       In* __restrict__ z, const double* __restrict__ kw_bar,
                                                       const double* __restrict__ kz_bar) {
  constexpr int NP = 16 * T;
  constexpr int KQ = 2 * NP / 4;
  const int i = blockIdx.y;
  const int64_t nn = (int64_t)nv * nv;
  const double* kwb = kw_bar + i * nn;
  const double* kzb = kz_bar + i * nn;
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
    for (int s0 = 0; s0 < KQ; s0 += 8) {
      In av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = 4 * (s0 + u) + (lane >> 4);
        In v = (In)0;
        if (rok && q < 2 * nv) v = (q < nv) ? w[row * nv + q] : zi[row * nv + (q - nv)];
        av[u] = v;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = 4 * (s0 + u) + (lane >> 4);
        const double a = (double)av[u];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int c = 16 * t + (lane & 15);
          double bv = 0.0;
          if (c < nv && q < 2 * nv) bv = (q < nv) ? kwb[(int64_t)q * nv + c] : 2.0 * kzb[(int64_t)(q - nv) * nv + c];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[t], 0, 0, 0);
        }
      }
    }
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
// One step of the reverse recurrence fused with the gradient on the pattern:
//
//   out = Lambda_k = a (A x) + b x + c xprev + d,   x = Lambda_{k+1}, xprev =
//         Lambda_{k+2}, d = Ybar_k, (a, b, c) = (2 alpha, 2 beta, -1);
//         x == NULL gives out = d (k = M), xprev == NULL drops the c term;
//   abar[p] += coef * Lambda_k[r] . y[c_p] for the stored entries p of row r,
//         y = Y_{k-1}, in FP64.
//
// A row of N_v values is held by L = N_v/4 lanes, 4 values each (16 bytes in FP32,
// 32 in FP64); a wave holds R = 64/L whole rows, so the L partial dot products of an
// entry are summed inside the wave with lane permutes.  Rows go to XCDs in contiguous
// ranges, as in the forward recurrence, and a lattice's rows are visited in the same tiled
// order (TILED); when a row fills a whole wave (WAVE_ROW: N_v = 256 in FP32) its CSR
// entries come through the scalar cache.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t lattice_row(int64_t rho, const RowOrder& o) {
  const int tile_rows = o.tx * o.ty;
  const int64_t col_rows = (int64_t)tile_rows * o.nz;
  const int tile = (int)(rho / col_rows);
  const int64_t rem = rho - (int64_t)tile * col_rows;
  const int z = (int)(rem / tile_rows);
  const int in = (int)(rem - (int64_t)z * tile_rows);
  const int yy = in / o.tx, xx = in - yy * o.tx;
  const int tiles_x = o.nx / o.tx;
  const int ty_i = tile / tiles_x, tx_i = tile - ty_i * tiles_x;
  return (int64_t)(tx_i * o.tx + xx) + (int64_t)o.nx * ((int64_t)(ty_i * o.ty + yy) + (int64_t)o.ny * z);
}

__device__ __forceinline__ double row_sum(double s, int lane, int q, int L) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double t = __shfl(s, (lane + off) & 63);
    if (q < off && q + off < L) s += t;
  }
  return s;  // the row's total, in its lane q == 0
}

template <typename T, typename V, bool TILED, bool WAVE_ROW>
__global__ void __launch_bounds__(256) reverse_step_kernel(int64_t n, int L, int R, int64_t nblocks, int64_t per_xcd,
                                                           const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col_idx,
                                                           const T* __restrict__ val, T a, T b, T c,
                                                           const V* __restrict__ x, const V* __restrict__ xprev,
                                                           const V* __restrict__ d, V* __restrict__ out,
                                                           const V* __restrict__ y, double coef,
                                                           double* __restrict__ abar, RowOrder order) {
  const int64_t lblock = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lblock >= nblocks) return;  // uniform over the workgroup
  const int lane = threadIdx.x & 63;
  const int g = lane / L;
  const int q = lane - g * L;
  const int64_t rho = (lblock * 4 + (threadIdx.x >> 6)) * R + g;
  const bool active = g < R && rho < n;
  int64_t rs = active ? (TILED ? lattice_row(rho, order) : rho) : 0;  // idle lanes read row 0 and write nothing
  if constexpr (WAVE_ROW) rs = __builtin_amdgcn_readfirstlane((int)rs);  // one row per wave
  const int p0 = row_ptr[rs];
  const int len = active ? row_ptr[rs + 1] - p0 : 0;
  const int64_t own = rs * L + q;
  V res;
  if (x) {
    V acc = (V)(T)0;
    for (int p = 0; p < len; p += 8) {
      int cols[8];
      T vals[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const bool ok = p + j < len;
        cols[j] = ok ? col_idx[p0 + p + j] : (int)rs;
        vals[j] = ok ? val[p0 + p + j] : (T)0;
      }
      V gv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {  // padded slots issue no gather
        if (p + j < len)
          gv[j] = x[(int64_t)cols[j] * L + q];
        else
          gv[j] = (V)(T)0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += vals[j] * gv[j];
    }
    res = a * acc + b * x[own];
    // Lambda_{k+2} and Ybar_k are read for the last time and Lambda_k is next read by the
    // following step's gathers: streamed with non-temporal hints, as in the forward
    // recurrence (175 -> 166 ms for the 1000 steps at N = 262144, N_v = 80)
    if (xprev) res += c * __builtin_nontemporal_load(&xprev[own]);
    res += __builtin_nontemporal_load(&d[own]);
  } else {
    res = __builtin_nontemporal_load(&d[own]);
  }
  if (active) __builtin_nontemporal_store(res, &out[own]);
  // every lane of the wave runs the permutes: the loop bound is the wave's longest row
  for (int j = 0; __any(j < len); j += 4) {
    int cols[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) cols[u] = (j + u < len) ? col_idx[p0 + j + u] : (int)rs;
    V yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (j + u < len)
        yv[u] = y[(int64_t)cols[u] * L + q];
      else
        yv[u] = (V)(T)0;
    }
    double sum[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double t = (double)res.x * (double)yv[u].x;
      t += (double)res.y * (double)yv[u].y;
      t += (double)res.z * (double)yv[u].z;
      t += (double)res.w * (double)yv[u].w;
      sum[u] = row_sum(t, lane, q, L);
    }
    if (q == 0 && active) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j + u < len) abar[p0 + j + u] += coef * sum[u];
    }
  }
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
hipError_t launch_zbar_big(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kwb,
                           const double* kzb, hipStream_t stream) {
  dim3 grid((unsigned)((n + ZB_ROWS_PER_BLOCK - 1) / ZB_ROWS_PER_BLOCK), ntb);
  if (is_f32)
    hipLaunchKernelGGL((zbar_big_kernel<T, float>), grid, dim3(256), 0, stream, n, nv, (const float*)w, (float*)z, kwb,
                       kzb);
  else
    hipLaunchKernelGGL((zbar_big_kernel<T, double>), grid, dim3(256), 0, stream, n, nv, (const double*)w, (double*)z,
                       kwb, kzb);
  return hipGetLastError();
}

template <int T>
hipError_t launch_zbar_t(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kwb,
                         const double* kzb, hipStream_t stream) {
  const size_t lds = (size_t)2 * (16 * T) * (16 * T) * sizeof(double);
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

// Split tables of the transposed sweep: rows k, columns the sweep points i,
// chi[k*ldk + i] = bf16(c[k][i]), clo = bf16(c[k][i] - chi), each rounded once from
// the FP64 value (ties to even); zero padding up to ldk.
__global__ void __launch_bounds__(256) split_rows_kernel(const double* __restrict__ c, int64_t ldc, int nt, int m1,
                                                         __bf16* __restrict__ chi, __bf16* __restrict__ clo,
                                                         int64_t ldk) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)m1 * ldk) return;
  const int k = (int)(gid / ldk);
  const int i = (int)(gid - (int64_t)k * ldk);
  __bf16 hi = (__bf16)0.f, lo = (__bf16)0.f;
  if (i < nt) {
    const double v = c[(int64_t)k * ldc + i];
    hi = (__bf16)v;
    lo = (__bf16)(v - (double)hi);
  }
  chi[gid] = hi;
  clo[gid] = lo;
}

}  // namespace

hipError_t launch_split_rows(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo, int64_t ldk,
                             hipStream_t stream) {
  const int64_t total = (int64_t)m1 * ldk;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, c, ldc, nt, m1,
                     chi, clo, ldk);
  return hipGetLastError();
}

hipError_t launch_zbar(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kw_bar,
                       const double* kz_bar, hipStream_t stream) {
  switch ((nv + 15) / 16) {
    case 1: return launch_zbar_t<1>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 2: return launch_zbar_t<2>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 3: return launch_zbar_t<3>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 4: return launch_zbar_t<4>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 5: return launch_zbar_t<5>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 6: return launch_zbar_t<6>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 7: case 8: return launch_zbar_big<8>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 9: case 10: case 11: case 12: return launch_zbar_big<12>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    case 13: case 14: case 15: case 16: return launch_zbar_big<16>(is_f32, n, nv, ntb, w, z, kw_bar, kz_bar, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, typename V>
hipError_t launch_reverse_t(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx, const T* val, T a,
                            T b, T c, const void* x, const void* xprev, const void* d, void* out, const void* y,
                            double coef, double* abar, const RowOrder& o, hipStream_t stream) {
  const int L = nv / 4;
  if (L < 1 || L > 64 || nv % 4) return hipErrorInvalidValue;
  const int R = 64 / L;
  const int64_t rows_per_block = 4 * (int64_t)R;
  const int64_t nblocks = (n + rows_per_block - 1) / rows_per_block;
  const int64_t per_xcd = (nblocks + 7) / 8;
  if (per_xcd * 8 > 0x7FFFFFFF) return hipErrorInvalidValue;
  const bool tiled = o.nx > 0;
  if (tiled && !(o.tx > 0 && o.ty > 0 && o.nx % o.tx == 0 && o.ny % o.ty == 0 && (int64_t)o.nx * o.ny * o.nz == n))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(per_xcd * 8)), block(256);
#define SSM_REVERSE_LAUNCH(TL, WR)                                                                                \
  hipLaunchKernelGGL((reverse_step_kernel<T, V, TL, WR>), grid, block, 0, stream, n, L, R, nblocks, per_xcd, row_ptr, \
                     col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, (const V*)y, coef,     \
                     abar, o)
  if (tiled && L == 64) SSM_REVERSE_LAUNCH(true, true);
  else if (tiled) SSM_REVERSE_LAUNCH(true, false);
  else if (L == 64) SSM_REVERSE_LAUNCH(false, true);
  else SSM_REVERSE_LAUNCH(false, false);
#undef SSM_REVERSE_LAUNCH
  return hipGetLastError();
}

hipError_t launch_transpose_coefficients(const double* c, int64_t ldc, int nt, int m1, double* ct64, float* ct32,
                                         int64_t ldct, hipStream_t stream) {
  const int64_t total = (int64_t)nt * ldct;
  hipLaunchKernelGGL(transpose_coefficients_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, c,
                     ldc, nt, m1, ct64, ct32, ldct);
  return hipGetLastError();
}

hipError_t launch_reverse_step_f64(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                   const double* val, double a, double b, double c, const double* x,
                                   const double* xprev, const double* d, double* out, const double* y, double coef,
                                   double* abar, hipStream_t stream, const RowOrder& order) {
  return launch_reverse_t<double, f64x4>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, y, coef, abar,
                                         order, stream);
}

hipError_t launch_reverse_step_f32(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                   const float* val, float a, float b, float c, const float* x, const float* xprev,
                                   const float* d, float* out, const float* y, double coef, double* abar,
                                   hipStream_t stream, const RowOrder& order) {
  return launch_reverse_t<float, f32x4>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, y, coef, abar,
                                        order, stream);
}

}  // namespace ssm
