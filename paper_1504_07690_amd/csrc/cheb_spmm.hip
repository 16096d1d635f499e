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
#include <algorithm>

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
// gathers of one row are in flight together; the slots past the row's end are masked
// off (a 7-entry stencil row issues 7 gathers, not 8).  The block read for the last
// time (xprev, d) is streamed with non-temporal hints.  The block written is stored
// normally when it takes at most 128 MiB, half of the 256 MB last-level cache: the next
// step gathers it and finds it there (an 84 MB FP32 block: 8% faster than a
// non-temporal store).  Larger blocks are stored non-temporally (a 168 MB FP64 block
// was 8% slower stored normally).
//
// out = a * (A x) + b * x + c * xprev + d   (xprev, d may be null; the reverse
// recurrence of the adjoint uses d for its direct seed).
//
// Rows of a lattice (row x + nx (y + ny z)) are visited tile by tile: tiles of tx x ty
// points of the x-y plane, each swept through every z, XCD x taking a contiguous eighth
// of the tiles.  The rows a stencil gathers for a tile's plane z are then the tile's planes
// z - 1, z, z + 1 and a one-point halo, a few hundred KB that the XCD's L2 keeps between
// the planes that reuse them; in plain row order the reuse spans two whole planes
// (16 MB at 128^2 points of 256 FP32 values), beyond the L2.
template <typename V>
__device__ __forceinline__ double vdot(const V& u, const V& v);
template <>
__device__ __forceinline__ double vdot<f32x4>(const f32x4& u, const f32x4& v) {
  return (double)u.x * (double)v.x + (double)u.y * (double)v.y + (double)u.z * (double)v.z + (double)u.w * (double)v.w;
}
template <>
__device__ __forceinline__ double vdot<f64x2>(const f64x2& u, const f64x2& v) {
  return u.x * v.x + u.y * v.y;
}

// DOTS: the workgroup also writes dots[2 lblock] = <out, x> and dots[2 lblock + 1] =
// <x, x> over its slices (FP64 sums of exact products), for the Chebyshev moments of
// Algorithm 2 by the product identity T_j T_k = (T_{j+k} + T_{|j-k|}) / 2.
// Workgroups of 256 lanes: 512 and 1024 gave the same time on a ring of blocks (each step
// reading the block the step before wrote), and 1024 slowed the FP64 and moment variants.
constexpr int CS_THREADS = 256;

// row visited at position rho of the tiled order
__device__ __forceinline__ int64_t tiled_row(int64_t rho, const RowOrder& o) {
  const int tile_rows = o.tx * o.ty;
  const int64_t col_rows = (int64_t)tile_rows * o.nz;  // a tile swept through every z
  const int tile = (int)(rho / col_rows);
  const int64_t rem = rho - (int64_t)tile * col_rows;
  const int z = (int)(rem / tile_rows);
  const int in = (int)(rem - (int64_t)z * tile_rows);
  const int yy = in / o.tx, xx = in - yy * o.tx;
  const int tiles_x = o.nx / o.tx;
  const int ty_i = tile / tiles_x, tx_i = tile - ty_i * tiles_x;
  return (int64_t)(tx_i * o.tx + xx) + (int64_t)o.nx * ((int64_t)(ty_i * o.ty + yy) + (int64_t)o.ny * z);
}

// WAVE_ROW (N_v elements of a row fill whole waves, 1 KB and more): the row index is the
// same on every lane of a wave, so its CSR entries are read through the scalar cache (one
// scalar load per entry or per 8 entries) instead of by 64 lanes reading the same address:
// a 27-point row then issues 27 vector gathers instead of 81 vector loads.
template <typename T, typename V, bool DOTS, bool KEEP, bool TILED, bool WAVE_ROW>
__global__ void __launch_bounds__(CS_THREADS) cheb_step_kernel(int64_t n, int nvv, int64_t nblocks, int64_t per_xcd,
                                                        const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        const T* __restrict__ val, T a, T b, T c,
                                                        const V* __restrict__ x, const V* __restrict__ xprev,
                                                        const V* __restrict__ d, V* __restrict__ out,
                                                        double* __restrict__ dots, RowOrder order) {
  const int64_t lblock = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lblock >= nblocks) return;  // uniform over the workgroup
  const int64_t gid0 = lblock * blockDim.x + threadIdx.x;
  const bool valid = gid0 < n * (int64_t)nvv;
  if (!DOTS && !valid) return;
  const int64_t vid = valid ? gid0 : 0;  // idle lanes of a DOTS block recompute slice 0 and store nothing
  const int64_t rho = vid / nvv;
  const int q = (int)(vid - rho * nvv);
  const int64_t r = TILED ? tiled_row(rho, order) : rho;
  const int64_t gid = r * nvv + q;
  V xp = (V)(T)0, dd = (V)(T)0;  // streamed operands first: they do not depend on the row's CSR
  if (xprev) xp = __builtin_nontemporal_load(&xprev[gid]);
  if (d) dd = __builtin_nontemporal_load(&d[gid]);
  V acc = (V)(T)0;
  if constexpr (WAVE_ROW) {
    const int ru = __builtin_amdgcn_readfirstlane((int)r);
    const int p0 = row_ptr[ru];
    const int p1 = row_ptr[ru + 1];
    for (int p = p0; p < p1; p += 8) {
      const int cnt = p1 - p;  // uniform
      int cols[8];
      T vals[8];
      if (cnt >= 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cols[j] = col_idx[p + j];
          vals[j] = val[p + j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          cols[j] = j < cnt ? col_idx[p + j] : ru;
          vals[j] = j < cnt ? val[p + j] : (T)0;
        }
      }
      V g[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) g[j] = (j < cnt) ? x[(int64_t)cols[j] * nvv + q] : (V)(T)0;
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += vals[j] * g[j];
    }
  } else {
  const int p0 = row_ptr[r];
  const int p1 = row_ptr[r + 1];
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
    for (int j = 0; j < 8; ++j) {  // padded slots issue no gather
      if (p + j < p1)
        g[j] = x[(int64_t)cols[j] * nvv + q];
      else
        g[j] = (V)(T)0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += vals[j] * g[j];
  }
  }
  const V xo = x[gid];
  V res = a * acc + b * xo;
  if (xprev) res += c * xp;
  if (d) res += dd;
  if (valid) {
    if constexpr (KEEP)
      out[gid] = res;
    else
      __builtin_nontemporal_store(res, &out[gid]);
  }
  if constexpr (DOTS) {
    __shared__ double red[2][CS_THREADS];
    red[0][threadIdx.x] = valid ? vdot<V>(res, xo) : 0.0;
    red[1][threadIdx.x] = valid ? vdot<V>(xo, xo) : 0.0;
    __syncthreads();
    for (int st = CS_THREADS / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) {
        red[0][threadIdx.x] += red[0][threadIdx.x + st];
        red[1][threadIdx.x] += red[1][threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      dots[2 * lblock] = red[0][0];
      dots[2 * lblock + 1] = red[1][0];
    }
  }
}

// Inner products of a group of recurrence steps from their workgroup partials: workgroup
// g reduces step s = s0 + g (partials at dots + 2 g nblocks) in a fixed order and writes
// sums[2 s] = <Y_s, Y_s> and sums[2 s + 1] = <Y_{s+1}, Y_s> (Y_0 = W).
__global__ void __launch_bounds__(256) moments_kernel(int64_t nblocks, const double* __restrict__ dots, int s0,
                                                      double* __restrict__ sums) {
  __shared__ double red[2][256];
  const double* d = dots + 2 * nblocks * (int64_t)blockIdx.x;
  double ox = 0.0, xx = 0.0;
  for (int64_t bidx = threadIdx.x; bidx < nblocks; bidx += 256) {
    ox += d[2 * bidx];
    xx += d[2 * bidx + 1];
  }
  red[0][threadIdx.x] = ox;
  red[1][threadIdx.x] = xx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int s = s0 + blockIdx.x;
    sums[2 * s] = red[1][0];
    sums[2 * s + 1] = red[0][0];
  }
}

// Algorithm 2 from the step inner products: T_s^2 = (T_{2s} + T_0)/2 and T_{s+1} T_s =
// (T_{2s+1} + T_1)/2 for symmetric A~ give N_v zeta_0 = <W, W>, N_v zeta_1 = <Y_1, W>,
// N_v zeta_l = 2 sums[l] - N_v zeta_{l mod 2} (l >= 2); then phi(t_i) = sum_l mu_l(t_i)
// zeta_l in a fixed order.  zeta (m1 doubles) may be NULL.
__global__ void __launch_bounds__(256) dgc_kernel(const double* __restrict__ c, int64_t ldc, int nt, int m1, int nv,
                                                  const double* __restrict__ sums, double* __restrict__ out,
                                                  double* __restrict__ zeta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double z0 = sums[0] / nv;
  const double z1 = m1 > 1 ? sums[1] / nv : 0.0;
  auto zl = [&](int l) { return l == 0 ? z0 : l == 1 ? z1 : 2.0 * sums[l] / nv - ((l & 1) ? z1 : z0); };
  if (zeta)
    for (int l = i; l < m1; l += gridDim.x * blockDim.x) zeta[l] = zl(l);
  if (i >= nt) return;
  double acc = 0.0;
  for (int l = 0; l < m1; ++l) acc += c[(int64_t)l * ldc + i] * zl(l);
  out[i] = acc;
}

// Box stencils.  Offset of lattice coordinate u2 from u1 on a periodic side of length m
// (m >= 3): -1, 0, 1, or 2 when u2 is farther away.
__device__ __forceinline__ int wrap_diff(int u1, int u2, int m) {
  int d = u2 - u1;
  if (d == m - 1) d = -1;
  if (d == 1 - m) d = 1;
  return (d >= -1 && d <= 1) ? d : 2;
}

// slot 9 (dz + 1) + 3 (dy + 1) + dx + 1 of entry (row, col) in the box of row's point, or -1
__device__ __forceinline__ int box_slot(int64_t row, int64_t col, int nx, int ny, int nz) {
  const int x1 = (int)(row % nx), y1 = (int)((row / nx) % ny), z1 = (int)(row / ((int64_t)nx * ny));
  const int x2 = (int)(col % nx), y2 = (int)((col / nx) % ny), z2 = (int)(col / ((int64_t)nx * ny));
  const int dx = wrap_diff(x1, x2, nx), dy = wrap_diff(y1, y2, ny), dz = wrap_diff(z1, z2, nz);
  if (dx == 2 || dy == 2 || dz == 2) return -1;
  return 9 * (dz + 1) + 3 * (dy + 1) + dx + 1;
}

__global__ void __launch_bounds__(256) box_check_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx, int nx, int ny, int nz,
                                                        int* __restrict__ bad) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  uint32_t seen = 0;
  for (int p = row_ptr[row]; p < row_ptr[row + 1]; ++p) {
    const int sl = box_slot(row, col_idx[p], nx, ny, nz);
    if (sl < 0 || (seen >> sl) & 1u) {
      *bad = 1;
      return;
    }
    seen |= 1u << sl;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) box_values_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col_idx,
                                                         const T* __restrict__ val, int nx, int ny, int nz,
                                                         T* __restrict__ box) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  T v[27];
#pragma unroll
  for (int s = 0; s < 27; ++s) v[s] = (T)0;
  for (int p = row_ptr[row]; p < row_ptr[row + 1]; ++p) {
    const int sl = box_slot(row, col_idx[p], nx, ny, nz);
#pragma unroll
    for (int s = 0; s < 27; ++s)
      if (s == sl) v[s] = val[p];
  }
#pragma unroll
  for (int s = 0; s < 27; ++s) box[row * 27 + s] = v[s];
}

// One step on a box stencil.  A wave computes kBoxRows consecutive points x0 .. x0 + R - 1
// of a tile row (one 64-lane slice of their N_v values): for each of the 9 lines (dy, dz)
// of their neighbourhood it gathers the R + 2 rows x0 - 1 .. x0 + R once and adds each
// point's three terms in the order dx = -1, 0, 1, so a point's terms are summed in box
// order (the CSR order of a row away from the lattice's wrap).  R + 2 gathers per line
// instead of 3 R; the values come through the scalar cache (the rows are wave-uniform).
template <typename T, typename V, bool KEEP>
__global__ void __launch_bounds__(CS_THREADS) box_step_kernel(int64_t n, int nvv, int64_t nwaves, int64_t nblocks,
                                                       int64_t per_xcd, const T* __restrict__ box, T a, T b,
                                                       T c, const V* __restrict__ x,
                                                       const V* __restrict__ xprev, const V* __restrict__ d,
                                                       V* __restrict__ out, RowOrder o) {
  constexpr int R = kBoxRows;
  const int64_t lblock = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lblock >= nblocks) return;
  const int64_t wid = lblock * (CS_THREADS / 64) + (threadIdx.x >> 6);
  if (wid >= nwaves) return;  // uniform over the wave; the kernel has no barrier
  const int lane = threadIdx.x & 63;
  const int wpr = nvv / 64;  // waves per row
  const int64_t g = wid / wpr;
  const int q = (int)(wid - g * wpr) * 64 + lane;
  const int r0 = __builtin_amdgcn_readfirstlane((int)tiled_row(g * R, o));
  const int nx = o.nx, ny = o.ny, nz = o.nz;
  const int x0 = r0 % nx, y = (r0 / nx) % ny, z = r0 / (nx * ny);
  V acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = (V)(T)0;
  const T* bx = box + (int64_t)r0 * 27;
  const int xl = x0 == 0 ? nx - 1 : x0 - 1;      // left neighbour of the first point
  const int xr = x0 + R == nx ? 0 : x0 + R;      // right neighbour of the last
#pragma unroll 1
  for (int dz = -1; dz <= 1; ++dz) {
    const int zz = z + dz < 0 ? nz - 1 : (z + dz == nz ? 0 : z + dz);
#pragma unroll 1
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = y + dy < 0 ? ny - 1 : (y + dy == ny ? 0 : y + dy);
      const int64_t line = (int64_t)nx * (yy + (int64_t)ny * zz);
      V gq[R + 2];
      gq[0] = x[(line + xl) * nvv + q];
#pragma unroll
      for (int i = 0; i < R; ++i) gq[i + 1] = x[(line + x0 + i) * nvv + q];
      gq[R + 1] = x[(line + xr) * nvv + q];
      const int so = 9 * (dz + 1) + 3 * (dy + 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r] += bx[27 * r + so] * gq[r];
        acc[r] += bx[27 * r + so + 1] * gq[r + 1];
        acc[r] += bx[27 * r + so + 2] * gq[r + 2];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t gid = (int64_t)(r0 + r) * nvv + q;
    V res = a * acc[r] + b * x[gid];
    if (xprev) res += c * __builtin_nontemporal_load(&xprev[gid]);
    if (d) res += __builtin_nontemporal_load(&d[gid]);
    if constexpr (KEEP)
      out[gid] = res;
    else
      __builtin_nontemporal_store(res, &out[gid]);
  }
}

template <typename T, typename V>
hipError_t launch_box(bool keep, int64_t n, int nvv, const T* box, T a, T b, T c, const T* x, const T* xprev,
                      const T* d, T* out, const RowOrder& o, hipStream_t stream) {
  const int64_t nwaves = n / kBoxRows * (nvv / 64);
  const int64_t nblocks = (nwaves + CS_THREADS / 64 - 1) / (CS_THREADS / 64);
  const int64_t per_xcd = (nblocks + 7) / 8;
  if (per_xcd * 8 > 0x7FFFFFFF || n > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(per_xcd * 8)), block(CS_THREADS);
  // The kernel uses no LDS; reserving 32 KB per workgroup caps residency at 5 workgroups (20
  // waves) per CU, so that the rows an XCD has in flight, 8 per wave with their neighbourhood
  // lines, stay near its 4 MB L2: at the 8 workgroups the registers allow they do not (27-point
  // 128^3 lattice, N_v = 256: 2.69 ms per step with 8, 2.12 with 4 or 5, 2.50 with 2 or 3).
  constexpr size_t kResidencyLds = 32 << 10;
  if (keep)
    hipLaunchKernelGGL((box_step_kernel<T, V, true>), grid, block, kResidencyLds, stream, n, nvv, nwaves, nblocks,
                       per_xcd, box, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, o);
  else
    hipLaunchKernelGGL((box_step_kernel<T, V, false>), grid, block, kResidencyLds, stream, n, nvv, nwaves, nblocks,
                       per_xcd, box, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, o);
  return hipGetLastError();
}

template <typename T, typename V, bool TILED, bool WR>
hipError_t launch_v(dim3 grid, bool keep, int64_t n, int nvv, int64_t nblocks, int64_t per_xcd, const int32_t* row_ptr,
                    const int32_t* col_idx, const T* val, T a, T b, T c, const T* x, const T* xprev, const T* d, T* out,
                    double* dots, const RowOrder& o, hipStream_t stream) {
  const dim3 block(CS_THREADS);
  if (dots && keep)
    hipLaunchKernelGGL((cheb_step_kernel<T, V, true, true, TILED, WR>), grid, block, 0, stream, n, nvv, nblocks, per_xcd,
                       row_ptr, col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, dots, o);
  else if (dots)
    hipLaunchKernelGGL((cheb_step_kernel<T, V, true, false, TILED, WR>), grid, block, 0, stream, n, nvv, nblocks, per_xcd,
                       row_ptr, col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, dots, o);
  else if (keep)
    hipLaunchKernelGGL((cheb_step_kernel<T, V, false, true, TILED, WR>), grid, block, 0, stream, n, nvv, nblocks, per_xcd,
                       row_ptr, col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out, nullptr, o);
  else
    hipLaunchKernelGGL((cheb_step_kernel<T, V, false, false, TILED, WR>), grid, block, 0, stream, n, nvv, nblocks,
                       per_xcd, row_ptr, col_idx, val, a, b, c, (const V*)x, (const V*)xprev, (const V*)d, (V*)out,
                       nullptr, o);
  return hipGetLastError();
}

template <typename T, typename V, int VEC>
hipError_t launch(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx, const T* val, T a, T b,
                  T c, const T* x, const T* xprev, const T* d, T* out, double* dots, const RowOrder& o,
                  hipStream_t stream) {
  const int nvv = nv / VEC;
  const int64_t threads = n * nvv;
  const int64_t nblocks = (threads + CS_THREADS - 1) / CS_THREADS;
  const int64_t per_xcd = (nblocks + 7) / 8;
  if (per_xcd * 8 > 0x7FFFFFFF) return hipErrorInvalidValue;
  // the written block is kept in the caches up to 128 MiB (see the store above)
  const bool keep = n * nv * (int64_t)sizeof(T) <= ((int64_t)128 << 20);
  const dim3 grid((unsigned)(per_xcd * 8));
  if (o.nx > 0) {
    if (!(o.tx > 0 && o.ty > 0 && o.nx % o.tx == 0 && o.ny % o.ty == 0 && (int64_t)o.nx * o.ny * o.nz == n))
      return hipErrorInvalidValue;
    if (o.box && !dots && nvv % 64 == 0 && o.tx % kBoxRows == 0 && o.nx >= 3 && o.ny >= 3 && o.nz >= 3)
      return launch_box<T, V>(keep, n, nvv, (const T*)o.box, a, b, c, x, xprev, d, out, o, stream);
    if (nvv % 64 == 0)
      return launch_v<T, V, true, true>(grid, keep, n, nvv, nblocks, per_xcd, row_ptr, col_idx, val, a, b, c, x, xprev,
                                        d, out, dots, o, stream);
    return launch_v<T, V, true, false>(grid, keep, n, nvv, nblocks, per_xcd, row_ptr, col_idx, val, a, b, c, x, xprev,
                                       d, out, dots, o, stream);
  }
  if (nvv % 64 == 0)
    return launch_v<T, V, false, true>(grid, keep, n, nvv, nblocks, per_xcd, row_ptr, col_idx, val, a, b, c, x, xprev,
                                       d, out, dots, o, stream);
  return launch_v<T, V, false, false>(grid, keep, n, nvv, nblocks, per_xcd, row_ptr, col_idx, val, a, b, c, x, xprev,
                                      d, out, dots, o, stream);
}

}  // namespace

hipError_t launch_cheb_step_f64(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* val, double a, double b, double c, const double* x,
                                const double* xprev, const double* d, double* out, hipStream_t stream,
                                double* dots, const RowOrder& order) {
  return launch<double, f64x2, 2>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, dots, order, stream);
}

hipError_t launch_cheb_step_f32(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const float* val, float a, float b, float c, const float* x,
                                const float* xprev, const float* d, float* out, hipStream_t stream,
                                double* dots, const RowOrder& order) {
  return launch<float, f32x4, 4>(n, nv, row_ptr, col_idx, val, a, b, c, x, xprev, d, out, dots, order, stream);
}

hipError_t launch_box_check(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int nx, int ny, int nz,
                            int* bad, hipStream_t stream) {
  if (nx < 3 || ny < 3 || nz < 3 || (int64_t)nx * ny * nz != n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(box_check_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, row_ptr, col_idx,
                     nx, ny, nz, bad);
  return hipGetLastError();
}

hipError_t launch_box_values(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* val, int is_f32,
                             int nx, int ny, int nz, void* box, hipStream_t stream) {
  if (nx < 3 || ny < 3 || nz < 3 || (int64_t)nx * ny * nz != n) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (is_f32)
    hipLaunchKernelGGL(box_values_kernel<float>, grid, block, 0, stream, n, row_ptr, col_idx, (const float*)val, nx, ny,
                       nz, (float*)box);
  else
    hipLaunchKernelGGL(box_values_kernel<double>, grid, block, 0, stream, n, row_ptr, col_idx, (const double*)val, nx,
                       ny, nz, (double*)box);
  return hipGetLastError();
}

int64_t cheb_step_blocks(int64_t n, int nv, int is_f32) {
  const int nvv = nv / (is_f32 ? 4 : 2);
  return (n * nvv + CS_THREADS - 1) / CS_THREADS;
}

hipError_t launch_moments(int64_t nblocks, const double* dots, int s0, int count, double* sums,
                          hipStream_t stream) {
  hipLaunchKernelGGL(moments_kernel, dim3((unsigned)count), dim3(256), 0, stream, nblocks, dots, s0, sums);
  return hipGetLastError();
}

hipError_t launch_dgc(const double* c, int64_t ldc, int nt, int m1, int nv, const double* sums, double* out,
                      double* zeta, hipStream_t stream) {
  hipLaunchKernelGGL(dgc_kernel, dim3((unsigned)((std::max(nt, m1) + 255) / 256)), dim3(256), 0, stream, c, ldc, nt,
                     m1, nv, sums, out, zeta);
  return hipGetLastError();
}

}  // namespace ssm
