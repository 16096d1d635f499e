// Gram matrices of the sweep (Eq. tracelr; Algorithm 5, step 13):
//
//   K_W(t_i) = W^T Z_i (symmetric),   K_Z(t_i) = Z_i^T Z_i,     Z_i, W: N x N_v
//
// in FP64 on v_mfma_f64_16x16x4_f64.  FP32 inputs are widened to FP64 exactly, so
// every product is exact and only the FP64 sums round.  W^T Z_i = W^T g(t_i I - A~) W is
// symmetric in exact arithmetic, so only its upper 16x16 blocks W_a^T Z_b (a <= b) are
// formed: a diagonal block is averaged with its transpose and the lower blocks mirror
// the upper ones.  This is one symmetric completion of the computed W^T Z; (W^T Z +
// Z^T W)/2 is another, with the same value in exact arithmetic and one more product.
//
// Work split (N_v <= 96): one workgroup per (sweep point, row segment); each of its
// four waves walks a contiguous quarter of the segment, four rows per MFMA step (the
// MFMA's k).  A wave keeps every upper 16x16 block (a <= b) of Z^T Z and of W^T Z in
// registers, so its operands come straight from memory: lane l reads column
// 16a + l%16 of row r + l/16 for each column block a, for Z_i and W (a 4-row slab is
// contiguous), two steps ahead of the MFMAs that consume them.  Each wave writes its
// partial blocks to scratch; a second kernel adds the partials in a fixed order and
// completes the symmetric matrices (deterministic).
#include "ssm_kernels.h"

namespace ssm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GR_WAVES = 4;

template <int T>
struct GramTiles {
  static constexpr int NPAIR = T * (T + 1) / 2;  // upper 16x16 blocks (a <= b)
};

template <int T, typename In>
struct GramStep {
  In z[T], w[T];
};

// Operand loads are buffer loads over the wave's own rows: the resource's byte range
// ends at the last row of the wave, and the hardware returns 0 for reads past it, so
// the rows of the last partial step arrive as zeros with no clamping, masking or
// branching.  Columns 16a + l%16 >= N_v of a row inside the range read the next row;
// they only feed output entries that are never stored.  Unpredicated loads whose
// values are used as loaded let the compiler count them: waiting for the oldest
// buffer does not also wait for the prefetch just issued.
template <typename In>
__device__ __forceinline__ In buffer_load(__amdgpu_buffer_rsrc_t r, int byte_off);
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer access (gfx9 family)

template <int T, typename In>
__device__ __forceinline__ void gram_load(GramStep<T, In>& st, __amdgpu_buffer_rsrc_t rz, __amdgpu_buffer_rsrc_t rw,
                                          int rel_row, int nv, const int (&lane_off)[T]) {
  const int base = rel_row * nv * (int)sizeof(In);
#pragma unroll
  for (int a = 0; a < T; ++a) {
    st.z[a] = buffer_load<In>(rz, base + lane_off[a]);
    st.w[a] = buffer_load<In>(rw, base + lane_off[a]);
  }
}

template <int T, typename In>
__global__ void __launch_bounds__(256) gram_kernel(int64_t n, int nv, int ntb, const In* __restrict__ w,
                                                   int64_t w_stride, const In* __restrict__ z, int64_t z_stride,
                                                   int64_t rows_per_seg, double* __restrict__ part) {
  using G = GramTiles<T>;
  const int i = blockIdx.x;
  const int seg = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: the buffer resources stay scalar
  const int64_t s_begin = (int64_t)seg * rows_per_seg;
  const int64_t s_end = (s_begin + rows_per_seg < n) ? s_begin + rows_per_seg : n;
  // contiguous quarter of the segment, a multiple of 4 rows
  int64_t q = (s_end - s_begin + GR_WAVES - 1) / GR_WAVES;
  q = (q + 3) / 4 * 4;
  const int64_t r_begin = s_begin + wave * q;
  const int64_t r_end = (r_begin + q < s_end) ? r_begin + q : s_end;
  const In* zi = z + (int64_t)i * z_stride;
  const In* wi = w + (int64_t)i * w_stride;
  const int rows = (int)((r_end > r_begin) ? r_end - r_begin : 0);
  const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(zi + (r_end > r_begin ? r_begin : 0) * nv), (short)0, rows * nv * (int)sizeof(In), kBufferWord3);
  const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(wi + (r_end > r_begin ? r_begin : 0) * nv), (short)0, rows * nv * (int)sizeof(In), kBufferWord3);
  int lane_off[T];
#pragma unroll
  for (int a = 0; a < T; ++a) lane_off[a] = ((lane >> 4) * nv + 16 * a + (lane & 15)) * (int)sizeof(In);

  f64x4 acc_zz[G::NPAIR], acc_wz[G::NPAIR];
#pragma unroll
  for (int p = 0; p < G::NPAIR; ++p) {
    acc_zz[p] = (f64x4){0.0, 0.0, 0.0, 0.0};
    acc_wz[p] = (f64x4){0.0, 0.0, 0.0, 0.0};
  }

  // two load buffers in rotation: each is refilled right after it is consumed with
  // the rows two steps (8 rows) ahead
  GramStep<T, In> buf0, buf1;
  // issue order buf0 then buf1, as in the loop, so the wait counts match on entry
  gram_load<T, In>(buf0, rz, rw, 0, nv, lane_off);
  __builtin_amdgcn_sched_barrier(0);
  gram_load<T, In>(buf1, rz, rw, 4, nv, lane_off);
  __builtin_amdgcn_sched_barrier(0);
  auto step = [&](GramStep<T, In>& b, int rr) {
    double zf[T], wf[T];
#pragma unroll
    for (int a = 0; a < T; ++a) {
      zf[a] = (double)b.z[a];
      wf[a] = (double)b.w[a];
    }
    gram_load<T, In>(b, rz, rw, rr + 8, nv, lane_off);
    // pair p = (a, b), a <= b, numbered row by row; fully unrolled, so every
    // operand and accumulator index is a compile-time constant
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int bb = a; bb < T; ++bb) {
        const int p = a * T - a * (a - 1) / 2 + (bb - a);
        acc_zz[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(zf[a], zf[bb], acc_zz[p], 0, 0, 0);
      }
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int bb = a; bb < T; ++bb) {
        const int p = a * T - a * (a - 1) / 2 + (bb - a);
        acc_wz[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(wf[a], zf[bb], acc_wz[p], 0, 0, 0);
      }
    __builtin_amdgcn_sched_barrier(0);  // keep steps apart: their operands need not be live together
  };
#pragma clang loop unroll(disable)
  for (int rr = 0; rr < rows; rr += 8) {
    step(buf0, rr);
    step(buf1, rr + 4);
  }

  // partial blocks -> scratch slot (seg, wave):
  // part[((slot*ntb + i)*2 + {0: ZZ, 1: WZ+ZW}) * nv*nv + row*nv + col]
  const int64_t nn = (int64_t)nv * nv;
  const int slot = seg * GR_WAVES + wave;
  double* pz = part + ((int64_t)slot * ntb + i) * 2 * nn;
  double* pw = pz + nn;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = a; b < T; ++b) {
      const int p = a * T - a * (a - 1) / 2 + (b - a);
      const int col = 16 * b + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * a + (lane >> 4) + 4 * r;  // FP64 result layout: D[l/16 + 4r][l%16]
        if (row < nv && col < nv) {
          pz[(int64_t)row * nv + col] = acc_zz[p][r];
          pw[(int64_t)row * nv + col] = acc_wz[p][r];
        }
      }
    }
}

// N_v above 96: the block grid is cut into tiles of 4 x 4 column blocks, (ti, tj) with
// ti <= tj, one tile per blockIdx.z; each wave keeps the 16 Z^T Z and 16 W^T Z
// blocks of its tile (on a diagonal tile the lower blocks are computed and not stored).
constexpr int GT_B = 4;

template <typename In>
struct GramTileStep {
  In za[GT_B], wa[GT_B], zb[GT_B];
};

template <typename In>
__device__ __forceinline__ void gram_tile_load(GramTileStep<In>& st, __amdgpu_buffer_rsrc_t rz,
                                               __amdgpu_buffer_rsrc_t rw, int rel_row, int nv,
                                               const int (&off_a)[GT_B], const int (&off_b)[GT_B]) {
  const int base = rel_row * nv * (int)sizeof(In);
#pragma unroll
  for (int a = 0; a < GT_B; ++a) {
    st.za[a] = buffer_load<In>(rz, base + off_a[a]);
    st.wa[a] = buffer_load<In>(rw, base + off_a[a]);
    st.zb[a] = buffer_load<In>(rz, base + off_b[a]);
  }
}

template <typename In>
__global__ void __launch_bounds__(256) gram_tiled_kernel(int64_t n, int nv, int ntb, const In* __restrict__ w,
                                                         int64_t w_stride, const In* __restrict__ z,
                                                         int64_t z_stride, int64_t rows_per_seg, int ntile,
                                                         double* __restrict__ part) {
  const int i = blockIdx.x;
  const int seg = blockIdx.y;
  // tile index -> (ti, tj), ti <= tj, row by row
  int ti = 0, rem = blockIdx.z;
  while (rem >= ntile - ti) {
    rem -= ntile - ti;
    ++ti;
  }
  const int tj = ti + rem;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t s_begin = (int64_t)seg * rows_per_seg;
  const int64_t s_end = (s_begin + rows_per_seg < n) ? s_begin + rows_per_seg : n;
  int64_t q = (s_end - s_begin + GR_WAVES - 1) / GR_WAVES;
  q = (q + 3) / 4 * 4;
  const int64_t r_begin = s_begin + wave * q;
  const int64_t r_end = (r_begin + q < s_end) ? r_begin + q : s_end;
  const In* zi = z + (int64_t)i * z_stride;
  const In* wi = w + (int64_t)i * w_stride;
  const int rows = (int)((r_end > r_begin) ? r_end - r_begin : 0);
  const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(zi + (r_end > r_begin ? r_begin : 0) * nv), (short)0, rows * nv * (int)sizeof(In), kBufferWord3);
  const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(wi + (r_end > r_begin ? r_begin : 0) * nv), (short)0, rows * nv * (int)sizeof(In), kBufferWord3);
  int off_a[GT_B], off_b[GT_B];
#pragma unroll
  for (int a = 0; a < GT_B; ++a) {
    off_a[a] = ((lane >> 4) * nv + 16 * (GT_B * ti + a) + (lane & 15)) * (int)sizeof(In);
    off_b[a] = ((lane >> 4) * nv + 16 * (GT_B * tj + a) + (lane & 15)) * (int)sizeof(In);
  }
  f64x4 acc_zz[GT_B * GT_B], acc_wz[GT_B * GT_B];
#pragma unroll
  for (int p = 0; p < GT_B * GT_B; ++p) {
    acc_zz[p] = (f64x4){0.0, 0.0, 0.0, 0.0};
    acc_wz[p] = (f64x4){0.0, 0.0, 0.0, 0.0};
  }
  GramTileStep<In> buf0, buf1;
  gram_tile_load<In>(buf0, rz, rw, 0, nv, off_a, off_b);
  __builtin_amdgcn_sched_barrier(0);
  gram_tile_load<In>(buf1, rz, rw, 4, nv, off_a, off_b);
  __builtin_amdgcn_sched_barrier(0);
  auto step = [&](GramTileStep<In>& b, int rr) {
    double za[GT_B], wa[GT_B], zb[GT_B];
#pragma unroll
    for (int a = 0; a < GT_B; ++a) {
      za[a] = (double)b.za[a];
      wa[a] = (double)b.wa[a];
      zb[a] = (double)b.zb[a];
    }
    gram_tile_load<In>(b, rz, rw, rr + 8, nv, off_a, off_b);
#pragma unroll
    for (int a = 0; a < GT_B; ++a)
#pragma unroll
      for (int bb = 0; bb < GT_B; ++bb) {
        const int p = a * GT_B + bb;
        acc_zz[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[a], zb[bb], acc_zz[p], 0, 0, 0);
        acc_wz[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[a], zb[bb], acc_wz[p], 0, 0, 0);
      }
    __builtin_amdgcn_sched_barrier(0);
  };
#pragma clang loop unroll(disable)
  for (int rr = 0; rr < rows; rr += 8) {
    step(buf0, rr);
    step(buf1, rr + 4);
  }
  const int64_t nn = (int64_t)nv * nv;
  const int slot = seg * GR_WAVES + wave;
  double* pz = part + ((int64_t)slot * ntb + i) * 2 * nn;
  double* pw = pz + nn;
#pragma unroll
  for (int a = 0; a < GT_B; ++a)
#pragma unroll
    for (int bb = 0; bb < GT_B; ++bb) {
      const int ab = GT_B * ti + a, bbl = GT_B * tj + bb;
      if (ab > bbl) continue;  // lower blocks of a diagonal tile
      const int p = a * GT_B + bb;
      const int col = 16 * bbl + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ab + (lane >> 4) + 4 * r;
        if (row < nv && col < nv) {
          pz[(int64_t)row * nv + col] = acc_zz[p][r];
          pw[(int64_t)row * nv + col] = acc_wz[p][r];
        }
      }
    }
}

// K(i)[r][c] = sum over segments of the stored upper block entry; the lower blocks
// mirror the upper ones; the diagonal blocks are averaged with their transpose (off the
// diagonal blocks o1 = o2, so the factor 1/2 leaves the entry as stored).
__global__ void __launch_bounds__(256) gram_reduce_kernel(int nv, int ntb, int nseg, const double* __restrict__ part,
                                                          double* __restrict__ k_w, double* __restrict__ k_z) {
  const int64_t nn = (int64_t)nv * nv;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ntb * nn) return;
  const int i = (int)(gid / nn);
  const int rc = (int)(gid - (int64_t)i * nn);
  const int r = rc / nv, c = rc % nv;
  const bool upper = (r >> 4) <= (c >> 4);
  const int64_t o1 = upper ? (int64_t)r * nv + c : (int64_t)c * nv + r;
  const bool lower = (c >> 4) <= (r >> 4);
  const int64_t o2 = lower ? (int64_t)c * nv + r : (int64_t)r * nv + c;
  double sz1 = 0.0, sw1 = 0.0, sz2 = 0.0, sw2 = 0.0;
  for (int s = 0; s < nseg; ++s) {
    const double* pz = part + ((int64_t)s * ntb + i) * 2 * nn;
    const double* pw = pz + nn;
    sz1 += pz[o1];
    sw1 += pw[o1];
    sz2 += pz[o2];
    sw2 += pw[o2];
  }
  k_z[gid] = 0.5 * (sz1 + sz2);
  k_w[gid] = 0.5 * (sw1 + sw2);
}

int64_t rows_per_segment(int64_t n, int nseg) {
  int64_t rps = (n + nseg - 1) / nseg;
  return (rps + 4 * GR_WAVES - 1) / (4 * GR_WAVES) * (4 * GR_WAVES);
}

template <int T>
hipError_t launch_t(int is_f32, int64_t n, int nv, int ntb, const void* w, int64_t ws, const void* z, int64_t zs,
                    int64_t rps, int segs, double* scratch, hipStream_t stream) {
  dim3 grid(ntb, segs);
  if (is_f32)
    hipLaunchKernelGGL((gram_kernel<T, float>), grid, dim3(64 * GR_WAVES), 0, stream, n, nv, ntb, (const float*)w, ws,
                       (const float*)z, zs, rps, scratch);
  else
    hipLaunchKernelGGL((gram_kernel<T, double>), grid, dim3(64 * GR_WAVES), 0, stream, n, nv, ntb,
                       (const double*)w, ws, (const double*)z, zs, rps, scratch);
  return hipGetLastError();
}

// Point i reads W at w + i * ws and Z at z + i * zs (elements).
hipError_t launch_strided(int is_f32, int64_t n, int nv, int ntb, const void* w, int64_t ws, const void* z,
                          int64_t zs, double* k_w, double* k_z, int nseg, double* scratch, hipStream_t stream) {
  // the number of segments actually used can drop when rows are rounded up
  const int64_t rps = rows_per_segment(n, nseg);
  const int segs = (int)((n + rps - 1) / rps);
  const int t = (nv + 15) / 16;
  // a wave's rows (plus the 8-row prefetch overrun) must be addressable by 32-bit byte offsets
  if ((rps / GR_WAVES + 16) * (int64_t)nv * (is_f32 ? 4 : 8) >= (int64_t)1 << 31) return hipErrorInvalidValue;
  hipError_t err;
  switch (t) {
    case 1: err = launch_t<1>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    case 2: err = launch_t<2>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    case 3: err = launch_t<3>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    case 4: err = launch_t<4>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    case 5: err = launch_t<5>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    case 6: err = launch_t<6>(is_f32, n, nv, ntb, w, ws, z, zs, rps, segs, scratch, stream); break;
    default: {
      if (t > 16) return hipErrorInvalidValue;
      const int ntile = (t + GT_B - 1) / GT_B;
      dim3 grid(ntb, segs, ntile * (ntile + 1) / 2);
      if (is_f32)
        hipLaunchKernelGGL(gram_tiled_kernel<float>, grid, dim3(64 * GR_WAVES), 0, stream, n, nv, ntb,
                           (const float*)w, ws, (const float*)z, zs, rps, ntile, scratch);
      else
        hipLaunchKernelGGL(gram_tiled_kernel<double>, grid, dim3(64 * GR_WAVES), 0, stream, n, nv, ntb,
                           (const double*)w, ws, (const double*)z, zs, rps, ntile, scratch);
      err = hipGetLastError();
    }
  }
  if (err != hipSuccess) return err;
  const int64_t total = (int64_t)ntb * nv * nv;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, nv, ntb,
                     segs * GR_WAVES, scratch, k_w, k_z);
  return hipGetLastError();
}

}  // namespace

int gram_scratch_slots(int nseg) { return nseg * GR_WAVES; }

hipError_t launch_gram(int is_f32, int64_t n, int nv, int ntb, const void* w, const void* z, double* k_w,
                       double* k_z, int nseg, double* scratch, hipStream_t stream) {
  return launch_strided(is_f32, n, nv, ntb, w, 0, z, n * nv, k_w, k_z, nseg, scratch, stream);
}

hipError_t launch_gram_pairs(int is_f32, int64_t n, int nv, int npairs, const void* y_hi, const void* y_lo,
                             int64_t stride, double* k_w, double* k_z, int nseg, double* scratch,
                             hipStream_t stream) {
  return launch_strided(is_f32, n, nv, npairs, y_hi, stride, y_lo, stride, k_w, k_z, nseg, scratch, stream);
}

}  // namespace ssm
