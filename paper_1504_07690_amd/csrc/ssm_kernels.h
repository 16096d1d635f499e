// Host-side launchers of the libssm kernels (internal to the library).
// Every launcher only enqueues on `stream` and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ssm {

// Algorithm 1 on the device (coeffs.hip).  c: (degree+1) x ldc doubles.
hipError_t launch_coefficients(double c0, double hw, double sigma, double inv_norm, const double* t, int nt,
                               int degree, int n_theta, double* c, float* c32, int64_t ldc, hipStream_t stream);
size_t coefficient_lds_bytes(int n_theta);
// Proposition 1: nu (2h+1 rows, row stride ldn, columns nt..ldn-1 zero) of the square of
// sum_{k<=h} mu_k T_k, mu read as rows 0..h of c (row stride ldc).
hipError_t launch_square_coefficients(const double* mu, int64_t ldc, int nt, int h, double* nu, int64_t ldn,
                                      hipStream_t stream);

// Philox4x32-10 + Box-Muller block (philox.hip).
hipError_t launch_gaussian_block(uint64_t seed, int64_t n, int nv, int dtype, void* w, hipStream_t stream);

// Visiting order of the rows of a lattice, rows x + nx (y + ny z) (nx = 0: plain row
// order): tiles of tx x ty points of the x-y plane (tx | nx, ty | ny), each through every z.
struct RowOrder {
  int nx = 0, ny = 0, nz = 0, tx = 0, ty = 0;
  // A's values in box order (launch_box_values), when every entry of a row lies in the
  // 3 x 3 x 3 box of its lattice point: the step then gathers each line of a neighbourhood
  // once for several rows (launch_cheb_step, no dots, rows of whole waves)
  const void* box = nullptr;
};
// Box stencils on a periodic nx x ny x nz lattice (each side >= 3): *bad = 1 if a row of the
// CSR has an entry outside the 3 x 3 x 3 box of its point or two entries in one box slot
// (bad is written only then); launch_box_values writes box[27 row + s], s = 9 (dz + 1) +
// 3 (dy + 1) + dx + 1, the value of the row's entry at that offset (0 where it has none).
hipError_t launch_box_check(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int nx, int ny, int nz,
                            int* bad, hipStream_t stream);
hipError_t launch_box_values(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const void* val, int is_f32,
                             int nx, int ny, int nz, void* box, hipStream_t stream);
// rows of a step computed together by the box kernel (tx must be a multiple of it)
constexpr int kBoxRows = 8;

// One Chebyshev step (cheb_spmm.hip):
//   out = a * (A x) + b * x + c * xprev + d   (xprev, d may be null)
// The rows are computed in `order` (the result does not depend on it).
hipError_t launch_cheb_step_f64(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* val, double a, double b, double c, const double* x,
                                const double* xprev, const double* d, double* out, hipStream_t stream,
                                double* dots = nullptr, const RowOrder& order = RowOrder{});
hipError_t launch_cheb_step_f32(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                const float* val, float a, float b, float c, const float* x,
                                const float* xprev, const float* d, float* out, hipStream_t stream,
                                double* dots = nullptr, const RowOrder& order = RowOrder{});
// Chebyshev moments for Algorithm 2.  With dots (2 cheb_step_blocks doubles) a step also
// writes workgroup partials of <out, x> and <x, x>.  launch_moments reduces `count`
// consecutive steps s0.. (partials 2 cheb_step_blocks apart; step s forms Y_{s+1} from
// Y_s) into sums[2s] = <Y_s, Y_s>, sums[2s+1] = <Y_{s+1}, Y_s>.  launch_dgc forms
// phi(t_i) = sum_l c[l][i] zeta_l (and zeta, if not NULL) from sums.
int64_t cheb_step_blocks(int64_t n, int nv, int is_f32);
hipError_t launch_moments(int64_t nblocks, const double* dots, int s0, int count, double* sums,
                          hipStream_t stream);
hipError_t launch_dgc(const double* c, int64_t ldc, int nt, int m1, int nv, const double* sums, double* out,
                      double* zeta, hipStream_t stream);

// Adjoint (adjoint.hip).
hipError_t launch_zbar(int is_f32, int64_t n, int nv, int ntb, const void* w, void* z, const double* kw_bar,
                       const double* kz_bar, hipStream_t stream);
// Reverse recurrence step fused with the gradient on the pattern of A:
// out = a (A x) + b x + c xprev + d (x NULL: out = d), then
// abar[p] += coef * out[r] . y[col[p]] for each stored entry p of each row r.
hipError_t launch_reverse_step_f64(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                   const double* val, double a, double b, double c, const double* x,
                                   const double* xprev, const double* d, double* out, const double* y, double coef,
                                   double* abar, hipStream_t stream, const RowOrder& order = RowOrder{});
hipError_t launch_reverse_step_f32(int64_t n, int nv, const int32_t* row_ptr, const int32_t* col_idx,
                                   const float* val, float a, float b, float c, const float* x, const float* xprev,
                                   const float* d, float* out, const float* y, double coef, double* abar,
                                   hipStream_t stream, const RowOrder& order = RowOrder{});
// chi[k*ldk + i] / clo: the BF16 split of c[k*ldc + i] (rows k < m1, points i < nt)
hipError_t launch_split_rows(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo, int64_t ldk,
                             hipStream_t stream);
hipError_t launch_transpose_coefficients(const double* c, int64_t ldc, int nt, int m1, double* ct64, float* ct32,
                                         int64_t ldct, hipStream_t stream);
// Sum of squares of `count` elements, two deterministic stages (reduce.hip).
// partial must hold reduce_partials() doubles; result written to *out (device).
int reduce_partials();
hipError_t launch_sumsq(const void* x, int64_t count, int is_f32, double* partial, double* out,
                        hipStream_t stream);

// Sweep GEMM (sweep_gemm.hip): z[i*e+q] (+)= sum_k c[k*ldc+i] y[k*e+q].
// acols: columns of c readable from the pointer (>= ntb, multiple of the vector width);
// c must be aligned to 16 bytes.
hipError_t launch_sweep_f64(int64_t e, int kc, int ntb, const double* c, int64_t ldc, int64_t acols,
                            const double* y, double* z, int accumulate, hipStream_t stream);
hipError_t launch_sweep_f32(int64_t e, int kc, int ntb, const float* c, int64_t ldc, int64_t acols,
                            const float* y, float* z, int accumulate, hipStream_t stream);
hipError_t launch_sweep_bf16(int64_t e, int kc, int ntb, const float* c, int64_t ldc, int64_t acols,
                             const float* y, float* z, int accumulate, hipStream_t stream);

// Split-BF16 sweep: chi/clo [i][ldk] (k contiguous, ldk % 8 == 0, 16-byte aligned rows),
// arows = rows of chi/clo readable from the pointers, a_elems = bf16 values readable from
// each pointer (at least (arows - 1) ldk + kc rounded up to 8: rows are read in 8-value
// pieces; reads past it return zeros).  e % 4 == 0, z 16-byte aligned.
// bstride != 16: the tables are in 16-degree blocks (launch_split_blocks): degree k of row
// i at (k / 16) bstride + 16 i + k % 16, with ldk = 16 and bstride >= 16 arows.
// k3: three products on the first k3 contraction indices of the launch (rounded up to
// whole 32-wide k-steps), Chi^T Yhi alone on the rest; k3 >= kc: three everywhere.
// m3: 256-row output tiles starting at or past row m3 take the single product
// throughout (m3 >= ntb: no such tile).
hipError_t launch_sweep_bf16x3(int64_t e, int kc, int ntb, const __bf16* chi, const __bf16* clo, int64_t ldk,
                               int64_t arows, int64_t a_elems, const float* y, float* z, int accumulate, int k3,
                               int m3, hipStream_t stream, int64_t bstride = 16);
size_t sweep_bf16x3_lds_bytes();
hipError_t launch_split_coefficients(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo,
                                     int64_t ldk, int ntp, hipStream_t stream);
// chi/clo in 16-degree blocks: degree k of point i at ((k / 16) ntp + i) 16 + k % 16, k < 16 nblk
hipError_t launch_split_blocks(const double* c, int64_t ldc, int nt, int m1, __bf16* chi, __bf16* clo, int nblk,
                               int ntp, hipStream_t stream);

// Gram (gram.hip).  scratch: gram_scratch_slots(nseg) * ntb * 2 * nv * nv doubles.
int gram_scratch_slots(int nseg);
hipError_t launch_gram(int is_f32, int64_t n, int nv, int ntb, const void* w, const void* z, double* k_w,
                       double* k_z, int nseg, double* scratch, hipStream_t stream);
// Pair mode: pair j takes W = y_hi + j*stride and Z = y_lo + j*stride (elements), so
// k_w[j] = (y_hi_j^T y_lo_j + y_lo_j^T y_hi_j)/2 and k_z[j] = y_lo_j^T y_lo_j.
hipError_t launch_gram_pairs(int is_f32, int64_t n, int nv, int npairs, const void* y_hi, const void* y_lo,
                             int64_t stride, double* k_w, double* k_z, int nseg, double* scratch,
                             hipStream_t stream);

// Algorithm 4 + trace (geneig.hip).
// Per-point FP64 scratch of launch_geneig_trace / launch_geneig_backward: the
// products, plus the two Jacobi matrices when N_v > 96 (they no longer fit in LDS).
// Jacobi matrices (n x (n+1) doubles each) held in LDS: both up to N_v = 96, the matrix
// being diagonalised alone up to N_v = 128 (its eigenvectors in global scratch), none above.
__host__ __device__ inline int geneig_lds_matrices(int nv) { return nv <= 96 ? 2 : nv <= 128 ? 1 : 0; }
__host__ __device__ inline int64_t geneig_scratch_doubles(int nv) {
  const int64_t n = nv;
  return n * n + (2 - geneig_lds_matrices(nv)) * n * (n + 1);
}
// Above N_v = 48 the trace (with or without the hybrid term) goes through a tridiagonal matrix
// (Householder reduction, QL for eig(K_W) with the eigenvectors built in LDS from a record
// of its rotations, bisection for eig(B)), kGeTriChunk points per launch group through
// geneig_tri_point_doubles of scratch each: 6 n^2 + 8 n + 8 (the reduced matrix, U^T, the
// rotation record of 4 n^2, the tridiagonal matrix and status).
constexpr int kGeTriChunk = 2048;
__host__ __device__ inline bool geneig_tri_path(int nv) { return nv > 48; }
__host__ __device__ inline int64_t geneig_tri_point_doubles(int nv) {
  const int64_t n = nv;
  return 6 * n * n + 8 * n + 8;
}
// FP64 scratch of launch_geneig_trace for ntb points
__host__ __device__ inline int64_t geneig_trace_scratch_doubles(int nv, int ntb) {
  if (geneig_tri_path(nv)) return (int64_t)(ntb < kGeTriChunk ? ntb : kGeTriChunk) * geneig_tri_point_doubles(nv);
  return (int64_t)ntb * geneig_scratch_doubles(nv);
}
__host__ __device__ inline int64_t geneig_backward_scratch_doubles(int nv) {
  const int64_t n = nv;
  return 3 * n * n + (2 - geneig_lds_matrices(nv)) * n * (n + 1);
}
// The backward on the tridiagonal path: the forward path's per-point scratch, then U^T and
// Kt (N_v^2 each), F(s), s, the kept indices and the point's state.
__host__ __device__ inline int64_t geneig_tri_bwd_point_doubles(int nv) {
  const int64_t n = nv;
  return geneig_tri_point_doubles(nv) + 2 * n * n + 4 * n + 8;
}
// FP64 scratch of launch_geneig_backward for ntb points
__host__ __device__ inline int64_t geneig_backward_scratch_total(int nv, int ntb) {
  if (geneig_tri_path(nv))
    return (int64_t)(ntb < kGeTriChunk ? ntb : kGeTriChunk) * geneig_tri_bwd_point_doubles(nv);
  return (int64_t)ntb * geneig_backward_scratch_doubles(nv);
}
// nvh > 0 adds the hybrid correction of Algorithm 6 from k_c (ntb x nvh x nv), trw (ntb)
// with hscr (ntb * nvh * nv doubles) as scratch.
// s_floor (ntb doubles, may be null): Algorithm 4 step 2 also drops s_j < s_floor[i].
// Point i writes r1 to ranks[i] and r2 to ranks[rank_stride + i] (rank_stride 0: ntb).
hipError_t launch_geneig_trace(int nv, int ntb, const double* k_w, const double* k_z, double g_max,
                               double tau, double rho, double* dos, int32_t* ranks, double* scratch,
                               hipStream_t stream, int nvh = 0, const double* k_c = nullptr,
                               const double* trw = nullptr, double* hscr = nullptr,
                               const double* s_floor = nullptr, int rank_stride = 0);
// RESS-DGC (ress.hip): X_l, l < m1, of the N_v' = nvp block from the pair Gram matrices,
// and the per-point split of K_mu, K_nu (nvp x nvp each) into K_W, K_Z (nv x nv), K_C
// (nvh x nv) and Tr K_W~.
hipError_t launch_ress_moments(int nvp, int m1, const double* pw, const double* pz, double* x, hipStream_t stream);
hipError_t launch_ress_extract(int nt, int nv, int nvh, const double* kmu, const double* knu, double* kw, double* kz,
                               double* kc, double* trw, hipStream_t stream);
// floor_out[i] = eta * sum_{l<=h} |mu_l(t_i)| max|X_l[:nv, :nv]| (xmax: h+1 doubles of scratch)
hipError_t launch_ress_floor(int nv, int nvp, int h, const double* x, const double* mu, int64_t ldc, int nt,
                             double eta, double* xmax, double* floor_out, hipStream_t stream);
size_t geneig_lds_bytes(int nv);
// Backward of Algorithm 4 (geneig.hip): kw_bar[i], kz_bar[i] = phibar[i] * d trace / d K_W, K_Z,
// the kept sets taken as in the forward kernel (s_floor as there, may be null).
// scratch: geneig_backward_scratch_total(nv, ntb) doubles.
hipError_t launch_geneig_backward(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                                  double rho, const double* phibar, double* kw_bar, double* kz_bar, double* scratch,
                                  hipStream_t stream, const double* s_floor = nullptr);
// Rounding floor of Algorithm 4's truncation for a sweep of limited precision:
// mun[i] = sqrt(sum_{l<m1} c[l*ldc + i]^2) (launch_coefficient_norms), then
// floor[i] = eta * mun[i] * (*w_sumsq) * inv_sqrt_e (launch_rounding_floor), with
// w_sumsq = ||W||_F^2 on the device and inv_sqrt_e = 1 / sqrt(N N_v).
// kmax[l] = max_{i < nt} |c[l*ldc + i]| for l < m1
hipError_t launch_coefficient_row_max(const double* c, int64_t ldc, int nt, int m1, double* kmax,
                                      hipStream_t stream);
hipError_t launch_coefficient_norms(const double* c, int64_t ldc, int nt, int m1, double* mun, hipStream_t stream);
hipError_t launch_rounding_floor(const double* mun, int nt, double eta, const double* w_sumsq, double inv_sqrt_e,
                                 double* floor_out, hipStream_t stream);

}  // namespace ssm
