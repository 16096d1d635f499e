// One step of the three-term Chebyshev recurrence on a block of N_v vectors
// (Algorithm 5, steps 9-10, with the rescaling of Section 2 folded in):
//
//   out = a * (A x) + b * x + c * xprev
//
// Y_1 = A~ Y_0 uses (a, b, c) = (alpha, beta, 0) and Y_{k+1} = 2 A~ Y_k - Y_{k-1} uses
// (2 alpha, 2 beta, -1), with A~ = alpha A + beta I, alpha = 2/(hi-lo),
// beta = -(hi+lo)/(hi-lo).  A~ is never formed.
//
// Layout: blocks are row-major N x N_v, so one row of the block is N_v contiguous
// values.  Each lane owns one 16-byte slice of one row (4 floats or 2 doubles):
// the lanes of a row read the row's CSR entries (the same addresses, merged by
// the memory pipeline) and gather the neighbours' slices, so every gathered row
// is read as whole 16-byte pieces of a contiguous N_v*elem segment.
#include "ssm_kernels.h"

namespace ssm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Rows are dealt to XCDs in contiguous ranges: workgroup b runs on XCD b % 8, so
// logical block (b % 8) * per_xcd + b / 8 gives XCD x the rows of blocks
// [x per_xcd, (x+1) per_xcd), swept in order.  A stencil neighbour a few planes
// away was then gathered by the same XCD shortly before, and is found in its L2.
// Up to 8 CSR entries of a row are fetched before their gathers are issued, so the
// gathers of one row are in flight together.  The block read once (xprev, d) and the
// block written are streamed with non-temporal hints, leaving the cache to the
// gathered block x.
//
// out = a * (A x) + b * x + c * xprev + d   (xprev, d may be null; the reverse
// recurrence of the adjoint uses d for its direct seed).
template <typename T, typename V>
__global__ void __launch_bounds__(256) cheb_step_kernel(int64_t n, int nvv, int64_t nblocks, int64_t per_xcd,
                                                        const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        const T* __restrict__ val, T a, T b, T c,
                                                        const V* __restrict__ x, const V* __restrict__ xprev,
                                                        const V* __restrict__ d, V* __restrict__ out) {
  const int64_t lblock = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lblock >= nblocks) return;
  const int64_t gid = lblock * blockDim.x + threadIdx.x;
  const int64_t r = gid / nvv;
  if (r >= n) return;
  const int q = (int)(gid - r * nvv);
  const int p0 = row_ptr[r];
  const int p1 = row_ptr[r + 1];
  V acc = (V)(T)0;
  for (int p = p0; p < p1; p += 8) {
    int cols[8];
    T vals[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool ok = p + j < p1;
      cols[j] = ok ? col_idx[p + j] : (int)r;
      vals[j] = ok ? val[p + j] : (T)0;
    }
    V g[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = x[(int64_t)cols[j] * nvv + q];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += vals[j] * g[j];
  }
  V res = a * acc + b * x[gid];
  if (xprev) res += c * __builtin_nontemporal_load(&xprev[gid]);
  if (d) res += __builtin_nontemporal_load(&d[gid]);
  __builtin_nontemporal_store(res, &out[gid]);
}

template <typename T, typename V, int VEC>
hipError_t launch(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx, const T* val, T a, T b,
                  T c, const T* x, const T* xprev, const T* d, T* out, hipStream_t stream) {
  const int nvv = nv / VEC;
  const int64_t threads = n * nvv;
  const int64_t nblocks = (threads + 255) / 256;
  const int64_t per_xcd = (nblocks + 7) / 8;
  if (per_xcd * 8 > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cheb_step_kernel<T, V>), dim3((unsigned)(per_xcd * 8)), dim3(256), 0, stream, n, nvv, nblocks,
                     per_xcd, row_ptr, col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cheb_step_f64(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* val, double a, double b, double c, const double* x,
                                const double* xprev, const double* d, double* out, hipStream_t stream) {
  return launch<double, f64x2, 2>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, stream);
}

hipError_t launch_cheb_step_f32(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const float* val, float a, float b, float c, const float* x,
                                const float* xprev, const float* d, float* out, hipStream_t stream) {
  return launch<float, f32x4, 4>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, stream);
}

}  // namespace ssm
