// The sweep of Algorithm 5 (steps 6-8) as a matrix product on the matrix cores.
//
// For a chunk of kc Chebyshev blocks Y_k = T_k(A~) W (each e = N*N_v contiguous
// values) and a batch of ntb sweep points:
//
//     Z_i[q] (+)= sum_k mu_k(t_i) Y_k[q]          i < ntb, q < e
//
// i.e. Z (ntb x e, row-major) = C^T (ntb x kc) * Y (kc x e, row-major), where the
// coefficient table C is stored k-major: C[k*ldc + i].  Both operands are read
// along their contiguous index, staged in LDS in [k][m] / [k][n] order, and fed to
// MFMA tiles.  Output tiles are (points x elements); a workgroup's tile pairs one
// slice of Y with many points, so each Y value fetched from memory serves BM points.
//
// XCD-aware order: workgroup b runs on XCD b % 8; the remap below gives every XCD
// a run of consecutive (point-tile, element-tile) pairs with the point tile
// fastest, so all point tiles that read one Y slice share that XCD's L2.
#include "ssm_kernels.h"

#include <type_traits>

namespace ssm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void tile_coords(int mt, int nt_tiles, int& m_tile, int& n_tile) {
  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int local = bid >> 3;
  m_tile = local % mt;
  n_tile = xcd + 8 * (local / mt);
  if (n_tile >= nt_tiles) n_tile = -1;
}

// ---------------------------------------------------------------------------
// FP32: v_mfma_f32_32x32x2_f32.  Tile 128 points x 128 elements x 16 k, four
// waves in a 2 x 2 arrangement, each wave 64 x 64 = 2 x 2 MFMA blocks.
// Operand lanes: a = A[m = lane%32][k = lane/32], b = B[k = lane/32][n = lane%32];
// result register r of lane l holds D[8(r/4) + 4(l/32) + r%4][l%32].
// ---------------------------------------------------------------------------
constexpr int F32_BM = 128, F32_BN = 128, F32_BK = 16, F32_PAD = 4;

__global__ void __launch_bounds__(256) sweep_f32_kernel(int64_t e, int kc, int ntb, const float* __restrict__ c,
                                                        int64_t ldc, int64_t acols, const float* __restrict__ y,
                                                        float* __restrict__ z, int accumulate, int mt,
                                                        int nt_tiles) {
  __shared__ float As[2][F32_BK][F32_BM + F32_PAD];
  __shared__ float Bs[2][F32_BK][F32_BN + F32_PAD];
  int m_tile, n_tile;
  tile_coords(mt, nt_tiles, m_tile, n_tile);
  if (n_tile < 0) return;
  const int64_t i0 = (int64_t)m_tile * F32_BM;
  const int64_t q0 = (int64_t)n_tile * F32_BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // global -> register staging: 2 float4 of A and 2 of B per thread
  f32x4 ra[2], rb[2];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = tid + 256 * u;
      const int kk = idx >> 5;
      const int c4 = (idx & 31) * 4;
      const int k = k0 + kk;
      f32x4 va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
      if (k < kc) {
        if (i0 + c4 < acols) va = *(const f32x4*)(c + (int64_t)k * ldc + i0 + c4);
        if (q0 + c4 < e) vb = *(const f32x4*)(y + (int64_t)k * e + q0 + c4);
      }
      ra[u] = va;
      rb[u] = vb;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = tid + 256 * u;
      const int kk = idx >> 5;
      const int c4 = (idx & 31) * 4;
      *(f32x4*)&As[buf][kk][c4] = ra[u];
      *(f32x4*)&Bs[buf][kk][c4] = rb[u];
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int nk = (kc + F32_BK - 1) / F32_BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tile((kt + 1) * F32_BK);
#pragma unroll
    for (int kk = 0; kk < F32_BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float a0 = As[buf][kr][wm * 64 + (lane & 31)];
      const float a1 = As[buf][kr][wm * 64 + 32 + (lane & 31)];
      const float b0 = Bs[buf][kr][wn * 64 + (lane & 31)];
      const float b1 = Bs[buf][kr][wn * 64 + 32 + (lane & 31)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t col = q0 + wn * 64 + b * 32 + (lane & 31);
      if (col >= e) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = i0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < ntb) {
          float* p = z + row * e + col;
          *p = accumulate ? *p + acc[a][b][r] : acc[a][b][r];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4_f64.  Tile 128 points x 64 elements x 16 k, four
// waves stacked along the points, each wave 32 x 64 = 2 x 4 MFMA blocks.
// Operand lanes: a = A[m = lane%16][k = lane/16], b = B[k = lane/16][n = lane%16];
// result register r of lane l holds D[l/16 + 4r][l%16].
// ---------------------------------------------------------------------------
constexpr int F64_BM = 128, F64_BN = 64, F64_BK = 16, F64_PAD = 2;

__global__ void __launch_bounds__(256) sweep_f64_kernel(int64_t e, int kc, int ntb, const double* __restrict__ c,
                                                        int64_t ldc, int64_t acols, const double* __restrict__ y,
                                                        double* __restrict__ z, int accumulate, int mt,
                                                        int nt_tiles) {
  __shared__ double As[2][F64_BK][F64_BM + F64_PAD];
  __shared__ double Bs[2][F64_BK][F64_BN + F64_PAD];
  int m_tile, n_tile;
  tile_coords(mt, nt_tiles, m_tile, n_tile);
  if (n_tile < 0) return;
  const int64_t i0 = (int64_t)m_tile * F64_BM;
  const int64_t q0 = (int64_t)n_tile * F64_BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  f64x2 ra[4], rb[2];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // A: 16 x 128 doubles = 1024 double2
      const int idx = tid + 256 * u;
      const int kk = idx >> 6;
      const int c2 = (idx & 63) * 2;
      const int k = k0 + kk;
      f64x2 v = {0.0, 0.0};
      if (k < kc && i0 + c2 < acols) v = *(const f64x2*)(c + (int64_t)k * ldc + i0 + c2);
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {  // B: 16 x 64 doubles = 512 double2
      const int idx = tid + 256 * u;
      const int kk = idx >> 5;
      const int c2 = (idx & 31) * 2;
      const int k = k0 + kk;
      f64x2 v = {0.0, 0.0};
      if (k < kc && q0 + c2 < e) v = *(const f64x2*)(y + (int64_t)k * e + q0 + c2);
      rb[u] = v;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      *(f64x2*)&As[buf][idx >> 6][(idx & 63) * 2] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int idx = tid + 256 * u;
      *(f64x2*)&Bs[buf][idx >> 5][(idx & 31) * 2] = rb[u];
    }
  };

  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};

  const int nk = (kc + F64_BK - 1) / F64_BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tile((kt + 1) * F64_BK);
#pragma unroll
    for (int kk = 0; kk < F64_BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[buf][kr][wave * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kr][b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t col = q0 + b * 16 + (lane & 15);
      if (col >= e) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wave * 32 + a * 16 + (lane >> 4) + 4 * r;
        if (row < ntb) {
          double* p = z + row * e + col;
          *p = accumulate ? *p + acc[a][b][r] : acc[a][b][r];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 inputs, FP32 accumulation: v_mfma_f32_32x32x16_bf16.  Tile 128 x 128 x 32.
// Operand lanes hold 8 consecutive k: a = A[m = lane%32][k = 8(lane/32) + j],
// b = B[k = 8(lane/32) + j][n = lane%32]; the result layout is that of the FP32
// 32x32 MFMA.  C and Y arrive k-major, so the tiles are transposed into
// [m][k] / [n][k] order while being rounded to bfloat16 (nearest even).
// ---------------------------------------------------------------------------
constexpr int BF_BM = 128, BF_BN = 128, BF_BK = 32, BF_PADK = 8;

__global__ void __launch_bounds__(256) sweep_bf16_kernel(int64_t e, int kc, int ntb, const float* __restrict__ c,
                                                         int64_t ldc, int64_t acols, const float* __restrict__ y,
                                                         float* __restrict__ z, int accumulate, int mt,
                                                         int nt_tiles) {
  __shared__ __bf16 As[BF_BM][BF_BK + BF_PADK];
  __shared__ __bf16 Bs[BF_BN][BF_BK + BF_PADK];
  int m_tile, n_tile;
  tile_coords(mt, nt_tiles, m_tile, n_tile);
  if (n_tile < 0) return;
  const int64_t i0 = (int64_t)m_tile * BF_BM;
  const int64_t q0 = (int64_t)n_tile * BF_BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  f32x4 ra[4], rb[4];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // 32 x 128 floats = 1024 float4 per operand
      const int idx = tid + 256 * u;
      const int kk = idx >> 5;
      const int c4 = (idx & 31) * 4;
      const int k = k0 + kk;
      f32x4 va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
      if (k < kc) {
        if (i0 + c4 < acols) va = *(const f32x4*)(c + (int64_t)k * ldc + i0 + c4);
        if (q0 + c4 < e) vb = *(const f32x4*)(y + (int64_t)k * e + q0 + c4);
      }
      ra[u] = va;
      rb[u] = vb;
    }
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = tid + 256 * u;
      const int kk = idx >> 5;
      const int c4 = (idx & 31) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        As[c4 + j][kk] = (__bf16)ra[u][j];
        Bs[c4 + j][kk] = (__bf16)rb[u][j];
      }
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int nk = (kc + BF_BK - 1) / BF_BK;
  load_tile(0);
  for (int kt = 0; kt < nk; ++kt) {
    store_tile();
    __syncthreads();
    if (kt + 1 < nk) load_tile((kt + 1) * BF_BK);
#pragma unroll
    for (int kk = 0; kk < BF_BK; kk += 16) {
      const int kb = kk + 8 * (lane >> 5);
      const bf16x8 a0 = *(const bf16x8*)&As[wm * 64 + (lane & 31)][kb];
      const bf16x8 a1 = *(const bf16x8*)&As[wm * 64 + 32 + (lane & 31)][kb];
      const bf16x8 b0 = *(const bf16x8*)&Bs[wn * 64 + (lane & 31)][kb];
      const bf16x8 b1 = *(const bf16x8*)&Bs[wn * 64 + 32 + (lane & 31)][kb];
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t col = q0 + wn * 64 + b * 32 + (lane & 31);
      if (col >= e) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = i0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < ntb) {
          float* p = z + row * e + col;
          *p = accumulate ? *p + acc[a][b][r] : acc[a][b][r];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Split BF16 ("bf16x3", Henry, Tang & Heinecke, ARITH 2019): every FP32 operand x
// is written as hi + lo with hi = bf16(x), lo = bf16(x - hi) (both round to nearest
// even), and C^T Y ~= Chi^T Yhi + Chi^T Ylo + Clo^T Yhi on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation: about 16 mantissa bits per product at BF16 matrix rate.
//
// Tile 256 points x 256 elements x 32 k, eight waves (2 x 4), each 128 x 64 = 4 x 2
// MFMA blocks (128 accumulators, so two waves share a SIMD).  The coefficients
// arrive pre-split in k-contiguous tables chi/clo [i][ldk]; the Y tile is split in
// registers while being transposed (a thread reads 8 consecutive k of 2 elements and
// writes, per element, 8 k of hi and of lo as 16-byte LDS stores).  LDS holds two stages
// of the four 256 x 32 BF16 tiles (128 KB); rows are 64 bytes and the 16-byte k-chunk c
// of row r sits at chunk c ^ ((r >> 2) & 3).  Element r of the Y tile lives in row
// r ^ ((r >> 1) & 1): a store instruction (element 2t + c from lane t) then covers rows
// of both parities, which fall in different halves of the bank window, and an operand
// read covers the same rows as in element order, permuted within groups of four; the
// counters show no bank conflicts for either.  One barrier per 32-degree unit.
//
// Global loads go through buffer resources (a wave-uniform base and a 32-bit lane
// offset), which keeps 64-bit addresses out of the vector registers; where the offsets
// allow (28 e + 1024 < 2^31), the 8 degrees a wave loads per unit share one resource.
// Degrees past kc get no records and read as zeros, so the coefficients there (of the
// next chunk, or past the tables' end, which also read as zeros) meet exact zeros, and
// every unit takes the same code.  The three-product units load one unit ahead of the
// LDS store that consumes them; the single-product units load two units ahead into two
// alternating register sets, with no conditions inside their loop, so that the waits of
// a store cover only its own set's loads.
//
// ---------------------------------------------------------------------------
constexpr int X3_BM = 256, X3_BN = 256, X3_BK = 32;
constexpr int X3_TILE = 256 * X3_BK;  // bf16 per LDS tile
typedef float f32x2 __attribute__((ext_vector_type(2)));

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// element offset of 16-byte chunk c (0..3) of row r in a 256 x 32 tile
__device__ __forceinline__ int x3_off(int r, int c) { return r * X3_BK + ((c ^ ((r >> 2) & 3)) << 3); }
// LDS row of element r of the Y tile: lane t stores elements 2t + c (c = 0, 1) into rows
// 2t + (c ^ (t & 1)), so that each store instruction of a wave covers rows of both parities
__device__ __forceinline__ int x3_brow(int r) { return r ^ ((r >> 1) & 1); }

template <bool ROW8>
__global__ void __launch_bounds__(512) sweep_bf16x3_kernel(int64_t e, int kc, int ntb,
                                                           const __bf16* __restrict__ chi,
                                                           const __bf16* __restrict__ clo, int64_t rstride,
                                                           int64_t bstride, int64_t arows, int64_t a_elems,
                                                           const float* __restrict__ y,
                                                           float* __restrict__ z, int accumulate, int mt,
                                                           int nt_tiles, int k3, int m3) {
  extern __shared__ __attribute__((aligned(16))) unsigned char x3_lds[];
  __bf16* lds = (__bf16*)x3_lds;
  int m_tile, n_tile;
  tile_coords(mt, nt_tiles, m_tile, n_tile);
  if (n_tile < 0) return;
  const int64_t i0 = (int64_t)m_tile * X3_BM;
  const int64_t q0 = (int64_t)n_tile * X3_BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;

  const int nu = (kc + X3_BK - 1) / X3_BK;
  const int nk3 = (k3 <= 0 || i0 >= m3) ? 0 : (k3 >= kc ? nu : (k3 + X3_BK - 1) / X3_BK);

  struct Staging {
    u16x8 ra_hi[2], ra_lo[2];
    f32x2 rb[8];
  };
  Staging S0, S1;
  const int c2 = (tid & 127) * 2;
  const int bch = __builtin_amdgcn_readfirstlane(tid >> 7);  // this wave's 8 degrees of B: 8 bch .. 8 bch + 7
  // Loads go through buffer resources: a lane adds a 32-bit byte offset to a wave-uniform
  // base.  Degrees past kc get a resource with no records, so their Y values read as zero
  // (the coefficients there are then multiplied by exact zeros); coefficient reads past the
  // end of the tables read as zero as well.
  const uint32_t boff = (uint32_t)(((q0 + c2 < e) ? c2 : e - 2 - q0) * 4);
  // ROW8 (28 e + 1024 < 2^31, so every offset fits in 31 bits): the 8 degrees a wave loads per
  // unit share one resource, and degree j of the 8 sits at byte offset 4 j e past the lane's.
  // The resource ends after the lane-clamped columns of the last degree below kc, so rows at or
  // past kc read zero, as with the per-degree resources.  One resource per 8 loads instead of
  // one per load removes about 30% of the kernel's scalar instructions, which the unit loops
  // issue between each barrier and the next MFMA phase (the sweep ran 8% faster).
  int boffj[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) boffj[j] = (int)boff + (ROW8 ? (int)(j * e * 4) : 0);
  // A lane loads 8 degrees (piece a_c of a row's 32): degrees 16 b .. 16 b + 15 of row i
  // sit at b bstride + i rstride (rows: rstride = ldk, bstride = 16; 16-degree blocks:
  // rstride = 16, bstride = 16 x rows)
  uint32_t aoff[2];
  const int a_c = tid & 3;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int piece = tid + 512 * h;
    const int64_t i = (i0 + (piece >> 2) < arows) ? i0 + (piece >> 2) : arows - 1;
    aoff[h] = (uint32_t)(((a_c >> 1) * bstride + i * rstride + (a_c & 1) * 8) * 2);
  }
  const int64_t abytes = a_elems * 2;  // the tables' extent from chi / clo
  auto rsrc = [](const void* p, int64_t bytes) {
    const int nrec = bytes <= 0 ? 0 : (bytes < 0x7FFFFFFF ? (int)bytes : 0x7FFFFFFF);
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, nrec, 0x00020000);
  };
  auto load_t = [&](Staging& S, int u, auto three) {
    constexpr bool THREE = decltype(three)::value;
    const int k0 = X3_BK * u;
    const int64_t ub = (int64_t)(k0 / 16) * bstride;  // the unit's first 16-degree block
    const auto rh = rsrc(chi + ub, abytes - ub * 2);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      S.ra_hi[h] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rh, (int)aoff[h], 0, 0));
    if constexpr (THREE) {
      const auto rl = rsrc(clo + ub, abytes - ub * 2);
#pragma unroll
      for (int h = 0; h < 2; ++h)
        S.ra_lo[h] = __builtin_bit_cast(u16x8, __builtin_amdgcn_raw_buffer_load_b128(rl, (int)aoff[h], 0, 0));
    }
    if constexpr (ROW8) {
      const int kb = k0 + 8 * bch;
      const int rows = kb < kc ? (kc - kb < 8 ? kc - kb : 8) : 0;
      const int64_t last = (e - q0) * 4 < 1024 ? (e - q0) * 4 : 1024;
      const auto rg = rsrc(y + (int64_t)(kb < kc ? kb : 0) * e + q0, rows ? (int64_t)(rows - 1) * e * 4 + last : 0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        S.rb[j] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rg, boffj[j], 0, 0));
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + 8 * bch + j;
        const auto rj = rsrc(y + (int64_t)(k < kc ? k : 0) * e + q0, k < kc ? 1024 : 0);
        S.rb[j] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rj, (int)boff, 0, 0));
      }
    }
  };
  auto load_unit = [&](Staging& S, int u) {
    if (u < nk3) load_t(S, u, std::true_type{});
    else load_t(S, u, std::false_type{});
  };
  auto store_t = [&](int st, int u, Staging& S, auto three) {
    constexpr bool THREE = decltype(three)::value;
    __bf16* ahi = lds + (4 * st + 0) * X3_TILE;
    __bf16* alo = lds + (4 * st + 1) * X3_TILE;
    __bf16* bhi = lds + (4 * st + 2) * X3_TILE;
    __bf16* blo = lds + (4 * st + 3) * X3_TILE;
    if (X3_BK * u + X3_BK > kc) {  // the unit that straddles kc: coefficients past it are not this chunk's
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (X3_BK * u + 8 * a_c + j >= kc) S.ra_hi[h][j] = S.ra_lo[h][j] = 0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int piece = tid + 512 * h;
      const int o = x3_off(piece >> 2, piece & 3);
      *(u16x8*)(ahi + o) = S.ra_hi[h];
      if constexpr (THREE) *(u16x8*)(alo + o) = S.ra_lo[h];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      bf16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 hh, ll;
        split_bf16(S.rb[j][c], hh, ll);
        h[j] = hh;
        l[j] = ll;
      }
      const int o = x3_off(x3_brow(c2 + c), bch);
      *(bf16x8*)(bhi + o) = h;
      if constexpr (THREE) *(bf16x8*)(blo + o) = l;
    }
  };
  auto store_unit = [&](int st, int u, Staging& S) {
    if (u < nk3) store_t(st, u, S, std::true_type{});
    else store_t(st, u, S, std::false_type{});
  };

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  auto mfma_step = [&](const __bf16* ahi, const __bf16* alo, const __bf16* bhi, const __bf16* blo, auto three) {
    constexpr bool THREE = decltype(three)::value;
    // raised issue priority over the MFMA phase: the SIMD's other wave, in its load and
    // store phase, then fills the gaps (1.6% faster at the default split, 2% single-product)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ch = 2 * ks + (lane >> 5);
      bf16x8 bh[2], bl[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int o = x3_off(x3_brow(wn * 64 + b * 32 + (lane & 31)), ch);
        bh[b] = *(const bf16x8*)(bhi + o);
        if constexpr (THREE) bl[b] = *(const bf16x8*)(blo + o);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int o = x3_off(wm * 128 + a * 32 + (lane & 31), ch);
        const bf16x8 ah = *(const bf16x8*)(ahi + o);
        if constexpr (THREE) {
          const bf16x8 al = *(const bf16x8*)(alo + o);
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[b], acc[a][b], 0, 0, 0);
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[b], acc[a][b], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
  };
  // Prefetch depth: the three-product units (three times the matrix work per unit) load one
  // unit ahead of the store that consumes it; the single-product units load two units ahead,
  // alternating between two register staging sets.
  load_unit(S0, 0);
  store_unit(0, 0, S0);
  if (nu > 1) load_unit(S0, 1);
  __syncthreads();
  int u = 0;
  // three-product units whose next two units are three-product units as well
  for (; u + 2 < nk3; ++u) {
    const __bf16* s = lds + 4 * (u & 1) * X3_TILE;
    mfma_step(s, s + X3_TILE, s + 2 * X3_TILE, s + 3 * X3_TILE, std::true_type{});
    store_t((u + 1) & 1, u + 1, S0, std::true_type{});
    __syncthreads();
    load_t(S0, u + 2, std::true_type{});
  }
  // the last (at most two) three-product units
  for (; u < nk3; ++u) {
    const __bf16* s = lds + 4 * (u & 1) * X3_TILE;
    mfma_step(s, s + X3_TILE, s + 2 * X3_TILE, s + 3 * X3_TILE, std::true_type{});
    if (u + 1 < nu) store_unit((u + 1) & 1, u + 1, S0);
    __syncthreads();
    if (u + 2 < nu) load_unit(S0, u + 2);
  }
  // single-product units: S0 holds unit u + 1, S1 takes unit u + 2
  load_t(S1, u + 2, std::false_type{});
  // No conditions inside the loop (units past the chunk load as zeros and are never read), so
  // that each store waits only for its own set's loads.
  auto tail_unit = [&](int u, Staging& Sn) {
    const __bf16* s = lds + 4 * (u & 1) * X3_TILE;
    mfma_step(s, s + X3_TILE, s + 2 * X3_TILE, s + 3 * X3_TILE, std::false_type{});
    store_t((u + 1) & 1, u + 1, Sn, std::false_type{});
    // keep the next unit's conversions below the barrier: hoisted above it, they would wait
    // for the loads issued one unit earlier
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    load_t(Sn, u + 3, std::false_type{});
  };
  for (; u + 1 < nu; u += 2) {
    tail_unit(u, S0);
    tail_unit(u + 1, S1);
  }
  if (u < nu) {
    const __bf16* s = lds + 4 * (u & 1) * X3_TILE;
    mfma_step(s, s + X3_TILE, s + 2 * X3_TILE, s + 3 * X3_TILE, std::false_type{});
  }

  // Epilogue through LDS, in four passes of 64 rows: the waves holding the pass's rows write
  // their accumulators to a 64 x 256 FP32 tile (rows padded by 4 floats), then every thread
  // stores 16-byte pieces of whole rows, so each store instruction of a wave covers one
  // contiguous 1 KB row segment of Z.
  float* zt = (float*)x3_lds;
  constexpr int ZLD = X3_BN + 4;
  __syncthreads();  // the last unit's operand reads are done
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    if (wm == (pass >> 1)) {
#pragma unroll
      for (int ah = 0; ah < 2; ++ah) {
        const int a = 2 * (pass & 1) + ah;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int col = wn * 64 + b * 32 + (lane & 31);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = ah * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            zt[row * ZLD + col] = acc[a][b][r];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int idx = tid + 512 * it;  // 64 rows x 64 pieces of 4 floats
      const int row = idx >> 6, c4 = (idx & 63) * 4;
      const int64_t grow = i0 + 64 * pass + row;
      const int64_t gcol = q0 + c4;
      if (grow < ntb && gcol < e) {
        const f32x4 v = *(const f32x4*)&zt[row * ZLD + c4];
        float* p = z + grow * e + gcol;
        if (gcol + 4 <= e) {
          // non-temporal: Z (84 GB at N = 262144, N_v = 80, N_t = 1000) is read back only by
          // the next kernel, long after it has left the caches; this was 1.6% faster with
          // three products on 268 degrees and 7% with one product everywhere
          if (accumulate) {
            const f32x4 old = *(const f32x4*)p;
            __builtin_nontemporal_store(old + v, (f32x4*)p);
          } else {
            __builtin_nontemporal_store(v, (f32x4*)p);
          }
        } else {
          for (int j = 0; j < 4 && gcol + j < e; ++j) p[j] = accumulate ? p[j] + v[j] : v[j];
        }
      }
    }
    __syncthreads();
  }
}

// chi/clo[i][k] = split of the FP64 coefficient c[k][i] (i < nt, k < m1), zero padded;
// each part is rounded once, from double, to the nearest bfloat16 (ties to even)
__global__ void __launch_bounds__(256) split_coefficients_kernel(const double* __restrict__ c, int64_t ldc, int nt,
                                                                 int m1, __bf16* __restrict__ chi,
                                                                 __bf16* __restrict__ clo, int64_t ldk, int ntp) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)ntp * ldk) return;
  const int i = (int)(gid / ldk);
  const int k = (int)(gid - (int64_t)i * ldk);
  __bf16 hi = (__bf16)0.f, lo = (__bf16)0.f;
  if (i < nt && k < m1) {
    const double v = c[(int64_t)k * ldc + i];
    hi = (__bf16)v;                 // one rounding, double -> bfloat16, nearest even
    lo = (__bf16)(v - (double)hi);  // the remainder, rounded the same way
  }
  chi[gid] = hi;
  clo[gid] = lo;
}

// The same split in 16-degree blocks: degree k of point i at ((k / 16) ntp + i) 16 + k % 16
// (blocks of ntp rows of 16, k < 16 nblk), so that the sweep's 256-point x 32-degree unit
// of a table is two runs of 256 x 32 bytes instead of 256 half-lines a row apart.
__global__ void __launch_bounds__(256) split_blocks_kernel(const double* __restrict__ c, int64_t ldc, int nt, int m1,
                                                           __bf16* __restrict__ chi, __bf16* __restrict__ clo,
                                                           int nblk, int ntp) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nblk * ntp * 16) return;
  const int kk = (int)(gid & 15);
  const int64_t row = gid >> 4;  // (k / 16) ntp + i
  const int b = (int)(row / ntp);
  const int i = (int)(row - (int64_t)b * ntp);
  const int k = 16 * b + kk;
  __bf16 hi = (__bf16)0.f, lo = (__bf16)0.f;
  if (i < nt && k < m1) {
    const double v = c[(int64_t)k * ldc + i];
    hi = (__bf16)v;
    lo = (__bf16)(v - (double)hi);
  }
  chi[gid] = hi;
  clo[gid] = lo;
}

template <typename T, typename K>
hipError_t launch_tiles(K kernel, int bm, int bn, int64_t e, int kc, int ntb, const T* c, int64_t ldc,
                        int64_t acols, const T* y, T* z, int accumulate, hipStream_t stream) {
  const int mt = (ntb + bm - 1) / bm;
  const int64_t ntiles = (e + bn - 1) / bn;
  const int64_t nt_pad = (ntiles + 7) / 8 * 8;
  const int64_t blocks = (int64_t)mt * nt_pad;
  if (blocks > 0x7FFFFFFF || ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, stream, e, kc, ntb, c, ldc, acols, y, z,
                     accumulate, mt, (int)ntiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_f32(int64_t e, int kc, int ntb, const float* c, int64_t ldc, int64_t acols, const float* y,
                            float* z, int accumulate, hipStream_t stream) {
  return launch_tiles(sweep_f32_kernel, F32_BM, F32_BN, e, kc, ntb, c, ldc, acols, y, z, accumulate, stream);
}

hipError_t launch_sweep_f64(int64_t e, int kc, int ntb, const double* c, int64_t ldc, int64_t acols,
                            const double* y, double* z, int accumulate, hipStream_t stream) {
  return launch_tiles(sweep_f64_kernel, F64_BM, F64_BN, e, kc, ntb, c, ldc, acols, y, z, accumulate, stream);
}

size_t sweep_bf16x3_lds_bytes() { return (size_t)2 * 4 * X3_TILE * sizeof(__bf16); }

hipError_t launch_sweep_bf16x3(int64_t e, int kc, int ntb, const __bf16* chi, const __bf16* clo, int64_t ldk,
                               int64_t arows, int64_t a_elems, const float* y, float* z, int accumulate, int k3,
                               int m3, hipStream_t stream, int64_t bstride) {
  const size_t lds = sweep_bf16x3_lds_bytes();
  const bool row8 = e * 4 * 7 + 1024 < ((int64_t)1 << 31);
  const void* kfn = row8 ? (const void*)sweep_bf16x3_kernel<true> : (const void*)sweep_bf16x3_kernel<false>;
  hipError_t err = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  const int mt = (ntb + X3_BM - 1) / X3_BM;
  const int64_t ntiles = (e + X3_BN - 1) / X3_BN;
  const int64_t nt_pad = (ntiles + 7) / 8 * 8;
  const int64_t blocks = (int64_t)mt * nt_pad;
  if (blocks > 0x7FFFFFFF || ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  // e % 4 == 0: 16-byte stores of Z rows; the tables' byte offsets are 32-bit resource offsets
  // bstride = 16: rows of ldk degrees; else blocks of 16 degrees, bstride apart, holding
  // rows of 16 (ldk = 16)
  if (bstride != 16 && (ldk != 16 || bstride < 16 * arows || bstride % 8)) return hipErrorInvalidValue;
  const int64_t plast = (kc + 7) / 8 - 1;  // the last 8-degree piece a row reads
  const int64_t need = (plast / 2) * bstride + (arows - 1) * ldk + (plast % 2) * 8 + 8;
  if (e < 4 || e % 4 || ((uintptr_t)z % 16) || arows < ntb || a_elems < need || a_elems * 2 > 0x7FFFFFFF)
    return hipErrorInvalidValue;
  if (row8)
    hipLaunchKernelGGL(sweep_bf16x3_kernel<true>, dim3((unsigned)blocks), dim3(512), lds, stream, e, kc, ntb, chi, clo,
                       ldk, bstride, arows, a_elems, y, z, accumulate, mt, (int)ntiles, k3, m3);
  else
    hipLaunchKernelGGL(sweep_bf16x3_kernel<false>, dim3((unsigned)blocks), dim3(512), lds, stream, e, kc, ntb, chi, clo,
                       ldk, bstride, arows, a_elems, y, z, accumulate, mt, (int)ntiles, k3, m3);
  return hipGetLastError();
}

hipError_t launch_split_coefficients(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo,
                                     int64_t ldk, int ntp, hipStream_t stream) {
  const int64_t total = (int64_t)ntp * ldk;
  hipLaunchKernelGGL(split_coefficients_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, c, ldc,
                     nt, m1, chi, clo, ldk, ntp);
  return hipGetLastError();
}

hipError_t launch_split_blocks(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo, int nblk,
                               int ntp, hipStream_t stream) {
  const int64_t total = (int64_t)nblk * ntp * 16;
  hipLaunchKernelGGL(split_blocks_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, c, ldc, nt,
                     m1, chi, clo, nblk, ntp);
  return hipGetLastError();
}

hipError_t launch_sweep_bf16(int64_t e, int kc, int ntb, const float* c, int64_t ldc, int64_t acols, const float* y,
                             float* z, int accumulate, hipStream_t stream) {
  return launch_tiles(sweep_bf16_kernel, BF_BM, BF_BN, e, kc, ntb, c, ldc, acols, y, z, accumulate, stream);
}

}  // namespace ssm
