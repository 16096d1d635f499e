// Gram matrices of the sweep (Eq. tracelr; Algorithm 5, step 13):
//
//   K_W(t_i) = (W^T Z_i + Z_i^T W) / 2,   K_Z(t_i) = Z_i^T Z_i,     Z_i, W: N x N_v
//
// in FP64 on v_mfma_f64_16x16x4_f64.  FP32 inputs are widened to FP64 exactly, so
// every product is exact and only the FP64 sums round.
//
// Work split: one workgroup per (sweep point, row segment).  A workgroup streams its
// rows through LDS, R rows at a time, as FP64 [row][col] tiles of Z_i and W padded
// to NP = 16*T columns.  Only the upper 16x16 blocks (a <= b) are formed: block
// (a, b) of Z^T Z, and block (a, b) of W^T Z + Z^T W as two MFMA chains into one
// accumulator.  The blocks are dealt round-robin to the four waves.  Each segment
// writes its partial blocks to scratch; a second kernel adds the segments in a
// fixed order, mirrors the lower triangle and halves K_W (deterministic).
#include "ssm_kernels.h"

namespace ssm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int GR_R = 32;  // rows per LDS stage (a multiple of the MFMA k = 4)

template <int T>
struct GramTiles {
  static constexpr int NP = 16 * T;
  static constexpr int NPAIR = T * (T + 1) / 2;
  static constexpr int PW = (NPAIR + 3) / 4;  // pairs per wave
};

template <int T, typename In>
__global__ void __launch_bounds__(256) gram_kernel(int64_t n, int nv, int ntb, const In* __restrict__ w,
                                                   const In* __restrict__ z, int64_t rows_per_seg,
                                                   double* __restrict__ part) {
  using G = GramTiles<T>;
  constexpr int LD = G::NP + 1;
  __shared__ double Zs[GR_R][LD];
  __shared__ double Ws[GR_R][LD];
  const int i = blockIdx.x;
  const int seg = blockIdx.y;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t r_begin = (int64_t)seg * rows_per_seg;
  const int64_t r_end = (r_begin + rows_per_seg < n) ? r_begin + rows_per_seg : n;
  const In* zi = z + (int64_t)i * n * nv;

  // this wave's pairs (a <= b), enumerated row by row of the upper triangle
  int pa[G::PW], pb[G::PW];
#pragma unroll
  for (int u = 0; u < G::PW; ++u) {
    const int pidx = wave + 4 * u;
    int a = 0, b = 0, cnt = 0;
    for (int aa = 0; aa < T; ++aa)
      for (int bb = aa; bb < T; ++bb) {
        if (cnt == pidx) { a = aa; b = bb; }
        ++cnt;
      }
    pa[u] = (pidx < G::NPAIR) ? a : -1;
    pb[u] = b;
  }

  f64x4 acc_zz[G::PW], acc_wz[G::PW];
#pragma unroll
  for (int u = 0; u < G::PW; ++u) {
    acc_zz[u] = (f64x4){0.0, 0.0, 0.0, 0.0};
    acc_wz[u] = (f64x4){0.0, 0.0, 0.0, 0.0};
  }

  // zero the padding columns once (the loads never touch them)
  for (int idx = tid; idx < GR_R * (LD - nv); idx += 256) {
    const int rr = idx / (LD - nv), cc = nv + idx % (LD - nv);
    Zs[rr][cc] = 0.0;
    Ws[rr][cc] = 0.0;
  }

  for (int64_t r0 = r_begin; r0 < r_end; r0 += GR_R) {
    const int rows = (r_end - r0 < GR_R) ? (int)(r_end - r0) : GR_R;
    __syncthreads();  // previous stage fully consumed
    // load rows [r0, r0+rows) of Z_i and W (contiguous), zero the missing rows
    const int nvec = GR_R * nv / 4;
    for (int idx = tid; idx < nvec; idx += 256) {
      const int flat = idx * 4;
      const int rr = flat / nv, cc = flat % nv;
      double zv[4] = {0.0, 0.0, 0.0, 0.0}, wv[4] = {0.0, 0.0, 0.0, 0.0};
      if (rr < rows) {
        const int64_t off = (r0 + rr) * nv + cc;
        if constexpr (sizeof(In) == 4) {
          const f32x4 a = *(const f32x4*)(zi + off);
          const f32x4 b = *(const f32x4*)(w + off);
#pragma unroll
          for (int j = 0; j < 4; ++j) { zv[j] = (double)a[j]; wv[j] = (double)b[j]; }
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const f64x2 a = *(const f64x2*)(zi + off + 2 * h);
            const f64x2 b = *(const f64x2*)(w + off + 2 * h);
            zv[2 * h] = a[0]; zv[2 * h + 1] = a[1];
            wv[2 * h] = b[0]; wv[2 * h + 1] = b[1];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Zs[rr][cc + j] = zv[j];
        Ws[rr][cc + j] = wv[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GR_R; kk += 4) {
      const int kr = kk + (lane >> 4);
      double zf[T], wf[T];
#pragma unroll
      for (int a = 0; a < T; ++a) {
        zf[a] = Zs[kr][16 * a + (lane & 15)];
        wf[a] = Ws[kr][16 * a + (lane & 15)];
      }
#pragma unroll
      for (int u = 0; u < G::PW; ++u) {
        if (pa[u] < 0) continue;
        double za = 0.0, zb = 0.0, wa = 0.0, wb = 0.0;
#pragma unroll
        for (int a = 0; a < T; ++a) {
          if (a == pa[u]) { za = zf[a]; wa = wf[a]; }
          if (a == pb[u]) { zb = zf[a]; wb = wf[a]; }
        }
        acc_zz[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(za, zb, acc_zz[u], 0, 0, 0);
        acc_wz[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, zb, acc_wz[u], 0, 0, 0);
        acc_wz[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(za, wb, acc_wz[u], 0, 0, 0);
      }
    }
  }

  // partial blocks -> scratch: part[((seg*ntb + i)*2 + {0: ZZ, 1: WZ+ZW}) * nv*nv + row*nv + col]
  const int64_t nn = (int64_t)nv * nv;
  double* pz = part + ((int64_t)seg * ntb + i) * 2 * nn;
  double* pw = pz + nn;
#pragma unroll
  for (int u = 0; u < G::PW; ++u) {
    if (pa[u] < 0) continue;
    const int col = 16 * pb[u] + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * pa[u] + (lane >> 4) + 4 * r;  // FP64 result layout: D[l/16 + 4r][l%16]
      if (row < nv && col < nv) {
        pz[(int64_t)row * nv + col] = acc_zz[u][r];
        pw[(int64_t)row * nv + col] = acc_wz[u][r];
      }
    }
  }
}

// K(i)[r][c] = sum over segments of the stored upper block entry; the lower blocks
// mirror the upper ones; the diagonal blocks are averaged with their transpose.
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
  k_w[gid] = 0.25 * (sw1 + sw2);
}

template <int T>
hipError_t launch_t(int is_f32, int64_t n, int nv, int ntb, const void* w, const void* z, int nseg,
                    double* scratch, hipStream_t stream) {
  int64_t rps = (n + nseg - 1) / nseg;
  rps = (rps + GR_R - 1) / GR_R * GR_R;
  const int segs = (int)((n + rps - 1) / rps);
  dim3 grid(ntb, segs);
  if (is_f32)
    hipLaunchKernelGGL((gram_kernel<T, float>), grid, dim3(256), 0, stream, n, nv, ntb, (const float*)w,
                       (const float*)z, rps, scratch);
  else
    hipLaunchKernelGGL((gram_kernel<T, double>), grid, dim3(256), 0, stream, n, nv, ntb, (const double*)w,
                       (const double*)z, rps, scratch);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gram(int is_f32, int64_t n, int nv, int ntb, const void* w, const void* z, double* k_w,
                       double* k_z, int nseg, double* scratch, hipStream_t stream) {
  // the number of segments actually used can drop when rows are rounded up
  int64_t rps = (n + nseg - 1) / nseg;
  rps = (rps + GR_R - 1) / GR_R * GR_R;
  const int segs = (int)((n + rps - 1) / rps);
  const int t = (nv + 15) / 16;
  hipError_t err;
  switch (t) {
    case 1: err = launch_t<1>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    case 2: err = launch_t<2>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    case 3: err = launch_t<3>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    case 4: err = launch_t<4>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    case 5: err = launch_t<5>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    case 6: err = launch_t<6>(is_f32, n, nv, ntb, w, z, nseg, scratch, stream); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  const int64_t total = (int64_t)ntb * nv * nv;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, nv, ntb,
                     segs, scratch, k_w, k_z);
  return hipGetLastError();
}

}  // namespace ssm
