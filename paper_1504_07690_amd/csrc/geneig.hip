// Algorithm 4 (truncated generalised eigenvalue problem) and the trace of
// Algorithm 5 (step 13), per sweep point, in FP64:
//
//   1. W^T Z = U S U^T                     (eigenvectors kept)
//   2. keep s_j >= tau max_i s_i            (nothing kept, trace 0, if max s <= 0)
//   3. B = S~^-1/2 U~^T (Z^T Z) U~ S~^-1/2,  eig(B) = xi   (values only)
//   4. keep xi in [0, (1 + rho) g_max], g_max = 1/(N sqrt(2 pi sigma^2))
//   trace = sum of kept xi, r1 = |kept s|, r2 = |kept xi|.
//
// Two eigensolvers.  Above N_v = 48 the trace (with or without the hybrid term of
// Algorithm 6) and its backward go through a tridiagonal matrix (Householder reduction;
// implicit QL for step 1, bisection or QL for step 3), in kernels per group of points
// (see geneig_tri_*).  At or below 48, and for points the QL gives up, one workgroup per
// point runs parallel cyclic Jacobi: sweeps in round-robin (tournament) order, so each round
// rotates N_v/2 disjoint index pairs at once: the pair angles are computed first
// (Golub & Van Loan, symmetric 2x2 Schur), then the rows of every pair are rotated,
// then the columns (and the eigenvector columns).  The pivot entries are set to
// exactly zero.  A sweep starts only while off(A)_F > 1e-14 ||A||_F.
// Jacobi's matrix and eigenvectors live in LDS for N_v <= 96 (2 * 96 * 97 doubles), the
// matrix alone up to N_v = 128 (eigenvectors in the point's global scratch), both in
// global scratch above that (N_v <= 256); the N_v x r1 product
// Z^T Z U~ S~^-1/2 goes through the same per-point scratch.
#include <type_traits>

#include "ssm_kernels.h"

namespace ssm {

namespace {

constexpr int GE_MAX_THREADS = 1024;
constexpr int GE_LDS_NV = 96;   // largest N_v whose two matrices sit in LDS (geneig_lds_matrices)
constexpr int GE_MAX_NV = 256;
constexpr int GE_MAX_SWEEPS = 40;

struct GeShared {
  double* A;      // n x ld
  double* V;      // n x ld
  double* s;      // eigenvalues
  double* scale;  // s^-1/2 of kept ones
  double* cs;     // pair cosines
  double* sn;     // pair sines
  double* red;    // reduction scratch (one double per thread)
  int* pp;        // pair rows
  int* qq;        // pair cols
  int* kidx;      // kept indices
  int* misc;      // [0] = r1
};

// Small arrays in LDS; A and V (n x (n+1) each) in LDS as geneig_lds_matrices says, the
// rest at `glob` (the point's global scratch).
__device__ void ge_layout(GeShared& sh, double* lds, int n, double* glob, int threads) {
  const int ld = n + 1;
  double* small = lds;
  const int mats = geneig_lds_matrices(n);
  if (mats == 0) {
    sh.A = glob;
    sh.V = glob + n * ld;
  } else if (mats == 1) {
    sh.A = lds;
    sh.V = glob;
    small = lds + n * ld;
  } else {
    sh.A = lds;
    sh.V = lds + n * ld;
    small = sh.V + n * ld;
  }
  sh.s = small;
  sh.scale = sh.s + GE_MAX_NV;
  sh.cs = sh.scale + GE_MAX_NV;
  sh.sn = sh.cs + GE_MAX_NV / 2;
  sh.red = sh.sn + GE_MAX_NV / 2;
  sh.pp = (int*)(sh.red + threads);
  sh.qq = sh.pp + GE_MAX_NV / 2;
  sh.kidx = sh.qq + GE_MAX_NV / 2;
  sh.misc = sh.kidx + GE_MAX_NV;
}

template <int TH>
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int st = TH / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Diagonalise the symmetric n x n matrix in sh.A (row stride ld); accumulate the
// rotations into V (if V != nullptr, V must hold the identity on entry).  V is kept
// transposed: eigenvector j is row j of the array (V[j * ld + r] is its entry r), so that
// a pair's rotation updates two contiguous rows.
// Each round rotates the disjoint index pairs (p_j, q_j) at once: A <- R^T A R, R the
// product of the pair rotations.  Entries of the 2 x 2 block of pairs (j, k) depend only
// on that block, so one lane updates a block (rows by pair j, then columns by pair k, the
// order of a row pass followed by a column pass) and writes it and its mirror (k, j),
// keeping A exactly symmetric; the pivot pair of a diagonal block becomes exactly 0.  When
// n is odd the index left without a partner forms a one-element pair (q = -1, no rotation).
template <int TH, int U>
__device__ void jacobi(const GeShared& sh, double* V, int n, int ld) {
  double* A = sh.A;
  const int tid = threadIdx.x;
  const int ne = n + (n & 1);
  const int npairs = ne / 2;
  const int nblocks = npairs * (npairs + 1) / 2;
  for (int sweep = 0; sweep < GE_MAX_SWEEPS; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int idx = tid; idx < n * n; idx += TH) {
      const int r = idx / n, c = idx - r * n;
      const double v = A[r * ld + c];
      all += v * v;
      if (r != c) off += v * v;
    }
    off = block_sum<TH>(off, sh.red);
    all = block_sum<TH>(all, sh.red);
    if (!(off > 1e-28 * all)) break;  // also stops on an all-zero matrix
    for (int round = 0; round < ne - 1; ++round) {
      if (tid < npairs) {
        const int s1 = tid, s2 = ne - 1 - tid;
        int p = (s1 == 0) ? 0 : 1 + (s1 - 1 + round) % (ne - 1);
        int q = 1 + (s2 - 1 + round) % (ne - 1);
        double c = 1.0, s = 0.0;
        if (p < n && q < n) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double app = A[p * ld + p], aqq = A[q * ld + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        } else {  // the phantom index n of an odd n: its partner stays as it is
          p = (p < n) ? p : q;
          q = -1;
        }
        sh.pp[tid] = p;
        sh.qq[tid] = q;
        sh.cs[tid] = c;
        sh.sn[tid] = s;
      }
      __syncthreads();
      // blocks (j, k), j <= k.  Each lane takes U blocks per pass and issues all their loads
      // before any store (the blocks of a round are disjoint), so that U loads are in flight
      // at once where A lives in global scratch.  In LDS (U = 1) the blocks are numbered row
      // by row of the triangle.  In global scratch a wave takes an 8 x 8 tile of blocks (j in
      // 8 consecutive pairs, k in 8 others): the entries it writes, and their mirrors, then
      // fall in 8 runs of 8 consecutive columns instead of 64 separate rows.
      const int T8 = (npairs + 7) / 8;
      const int nwork = U == 1 ? nblocks : T8 * (T8 + 1) / 2 * 64;
      // row j of a triangle of side P starts at j P - j (j - 1) / 2: the quadratic inverted in
      // float (within one of the row for P <= 128), then corrected by one step
      auto tri = [](int idx, int P, int& j, int& k) {
        const int P2 = 2 * P + 1;
        j = (int)((P2 - sqrtf((float)(P2 * P2 - 8 * idx))) * 0.5f);
        j = j < 0 ? 0 : (j >= P ? P - 1 : j);
        if (j * P - j * (j - 1) / 2 > idx)
          --j;
        else if ((j + 1) * P - (j + 1) * j / 2 <= idx)
          ++j;
        k = j + (idx - (j * P - j * (j - 1) / 2));
      };
      for (int i0 = tid; i0 < nwork; i0 += U * TH) {
        int jj[U], kk[U];
        double a[U], b[U], c0[U], d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = i0 + u * TH;
          jj[u] = -1;
          if (idx >= nwork) continue;
          int j, k;
          if (U == 1) {
            tri(idx, npairs, j, k);
          } else {  // TH is a multiple of 64: a wave's lanes share one tile
            int tj, tk;
            tri(idx >> 6, T8, tj, tk);
            j = 8 * tj + ((idx & 63) >> 3);
            k = 8 * tk + (idx & 7);
            if (j >= npairs || k >= npairs || j > k) continue;
          }
          const int pj = sh.pp[j], qj = sh.qq[j], pk = sh.pp[k], qk = sh.qq[k];
          if (qj < 0 || qk < 0) {  // a one-element pair: a row, a column or one entry
            if (qj < 0 && qk < 0) continue;  // its diagonal entry does not change
            // the single index x against the pair (y0, y1)
            const int x = qj < 0 ? pj : pk;
            const int y0 = qj < 0 ? pk : pj, y1 = qj < 0 ? qk : qj;
            a[u] = A[x * ld + y0];
            b[u] = A[x * ld + y1];
          } else {
            a[u] = A[pj * ld + pk];
            b[u] = A[pj * ld + qk];
            c0[u] = A[qj * ld + pk];
            d[u] = A[qj * ld + qk];
          }
          jj[u] = j;
          kk[u] = k;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = jj[u], k = kk[u];
          if (j < 0) continue;
          const int pj = sh.pp[j], qj = sh.qq[j], pk = sh.pp[k], qk = sh.qq[k];
          const double cj = sh.cs[j], sj = sh.sn[j], ck = sh.cs[k], sk = sh.sn[k];
          if (qj < 0 || qk < 0) {  // rotated by the pair's (c, s)
            const int x = qj < 0 ? pj : pk;
            const int y0 = qj < 0 ? pk : pj, y1 = qj < 0 ? qk : qj;
            const double c = qj < 0 ? ck : cj, s = qj < 0 ? sk : sj;
            const double n0 = c * a[u] - s * b[u], n1 = s * a[u] + c * b[u];
            A[x * ld + y0] = n0;
            A[x * ld + y1] = n1;
            A[y0 * ld + x] = n0;
            A[y1 * ld + x] = n1;
            continue;
          }
          // rows by pair j
          const double ra = cj * a[u] - sj * c0[u], rc = sj * a[u] + cj * c0[u];
          const double rb = cj * b[u] - sj * d[u], rd = sj * b[u] + cj * d[u];
          // columns by pair k
          const double na = ck * ra - sk * rb, nb = sk * ra + ck * rb;
          const double nc = ck * rc - sk * rd, nd = sk * rc + ck * rd;
          if (j == k) {  // the pivot pair becomes exactly 0
            A[pj * ld + pj] = na;
            A[qj * ld + qj] = nd;
            A[pj * ld + qj] = 0.0;
            A[qj * ld + pj] = 0.0;
          } else {
            A[pj * ld + pk] = na;
            A[pj * ld + qk] = nb;
            A[qj * ld + pk] = nc;
            A[qj * ld + qk] = nd;
            A[pk * ld + pj] = na;
            A[qk * ld + pj] = nb;
            A[pk * ld + qj] = nc;
            A[qk * ld + qj] = nd;
          }
        }
      }
      if (V) {  // V <- V R: columns of each pair, U entries per lane and pass as above
        for (int i0 = tid; i0 < npairs * n; i0 += U * TH) {
          int rr[U], kk[U];
          double vp[U], vq[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int idx = i0 + u * TH;
            kk[u] = -1;
            if (idx >= npairs * n) continue;
            const int k = idx / n, row = idx - k * n;
            const int p = sh.pp[k], q = sh.qq[k];
            if (q < 0) continue;
            vp[u] = V[p * ld + row];
            vq[u] = V[q * ld + row];
            kk[u] = k;
            rr[u] = row;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = kk[u];
            if (k < 0) continue;
            const int p = sh.pp[k], q = sh.qq[k], row = rr[u];
            const double c = sh.cs[k], s = sh.sn[k];
            V[p * ld + row] = c * vp[u] - s * vq[u];
            V[q * ld + row] = s * vp[u] + c * vq[u];
          }
        }
      }
      __syncthreads();
    }
  }
}

// Jacobi with the batching that suits where the matrices of a point with N_v = nv live:
// one entry per lane and pass when both are in LDS, four when either is in global scratch.
template <int TH>
__device__ void jacobi_for(const GeShared& sh, double* V, int m, int ld, int nv) {
  if (geneig_lds_matrices(nv) == 2)
    jacobi<TH, 1>(sh, V, m, ld);
  else
    jacobi<TH, 4>(sh, V, m, ld);
}

// Point i's scratch starts at scratch + i scr_stride.  With `only` set, point i is
// skipped unless only[i scr_stride] is 1 (the points the tridiagonal path gave up).
// With nvh > 0 (Algorithm 6 / 7 with N~_v = nvh columns of W~) the point also gets the
// hybrid correction (Tr K_W~ - ||K_C C~||_F^2) / N~_v, C~ = U~ S~^-1/2 Q~ with Q~ the
// eigenvectors of step 3 that pass step 4: G = K_C U~ S~^-1/2 (N~_v x r1, in hscr) is
// formed before V is reused for Q, then ||G Q~||_F^2 in a fixed order.
template <int TH>
__global__ void __launch_bounds__(TH) geneig_trace_kernel(int nv, const double* __restrict__ k_w,
                                                                  const double* __restrict__ k_z, double g_max,
                                                                  double tau, double rho, double* __restrict__ dos,
                                                                  int32_t* __restrict__ ranks, int rank_stride,
                                                                  double* __restrict__ scratch, int nvh,
                                                                  const double* __restrict__ k_c,
                                                                  const double* __restrict__ trw,
                                                                  double* __restrict__ hscr,
                                                                  const double* __restrict__ s_floor,
                                                                  int64_t scr_stride,
                                                                  const double* __restrict__ only) {
  extern __shared__ double lds[];
  const int n = nv;
  const int ld = n + 1;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (only && only[i * scr_stride] != 1.0) return;  // a point the tridiagonal path finished
  const double* kw = k_w + i * nn;
  const double* kz = k_z + i * nn;
  double* tmat = scratch + i * scr_stride;
  GeShared sh;
  ge_layout(sh, lds, n, tmat + nn, TH);

  for (int idx = tid; idx < n * n; idx += TH) {
    const int r = idx / n, c = idx - r * n;
    sh.A[r * ld + c] = kw[idx];
    sh.V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // 1. W^T Z = U S U^T
  jacobi_for<TH>(sh, sh.V, n, ld, n);
  for (int j = tid; j < n; j += TH) sh.s[j] = sh.A[j * ld + j];
  __syncthreads();

  // 2. truncation
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, sh.s[j]);
    int r1 = 0;
    if (smax > 0.0) {
      const double thr = s_floor ? fmax(tau * smax, s_floor[i]) : tau * smax;
      for (int j = 0; j < n; ++j)
        if (sh.s[j] >= thr) {
          sh.kidx[r1] = j;
          sh.scale[r1] = 1.0 / sqrt(sh.s[j]);
          ++r1;
        }
    }
    sh.misc[0] = r1;
  }
  __syncthreads();
  const int r1 = sh.misc[0];
  if (r1 == 0) {
    if (tid == 0) {
      dos[i] = nvh ? trw[i] / nvh : 0.0;  // C~ is empty: only Tr K_W~ / N~_v remains
      if (ranks) {
        ranks[i] = 0;
        ranks[rank_stride + i] = 0;
      }
    }
    return;
  }
  double* g = nvh ? hscr + (int64_t)i * nvh * nv : nullptr;
  if (nvh) {  // G = K_C U~ S~^-1/2  (N~_v x r1, row stride r1)
    const double* kci = k_c + (int64_t)i * nvh * nv;
    for (int idx = tid; idx < nvh * r1; idx += TH) {
      const int a = idx / r1, b = idx - a * r1;
      const int kb = sh.kidx[b];
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += kci[(int64_t)a * n + c] * sh.V[kb * ld + c];
      g[idx] = acc * sh.scale[b];
    }
  }

  // 3a. T = (Z^T Z) U~ S~^-1/2   (n x r1, global scratch, row stride r1)
  for (int idx = tid; idx < n * r1; idx += TH) {
    const int row = idx / r1, a = idx - row * r1;
    const int ka = sh.kidx[a];
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += kz[(int64_t)row * n + c] * sh.V[ka * ld + c];
    tmat[idx] = acc * sh.scale[a];
  }
  __threadfence_block();
  __syncthreads();
  // 3b. B = S~^-1/2 U~^T T  -> A (r1 x r1)
  for (int idx = tid; idx < r1 * r1; idx += TH) {
    const int a = idx / r1, b = idx - a * r1;
    const int ka = sh.kidx[a];
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += sh.V[ka * ld + c] * tmat[(int64_t)c * r1 + b];
    sh.A[a * ld + b] = acc * sh.scale[a];
  }
  __syncthreads();
  for (int idx = tid; idx < r1 * r1; idx += TH) {
    const int a = idx / r1, b = idx - a * r1;
    if (a < b) {
      const double m = 0.5 * (sh.A[a * ld + b] + sh.A[b * ld + a]);
      sh.A[a * ld + b] = m;
      sh.A[b * ld + a] = m;
    }
  }
  __syncthreads();
  if (nvh) {  // eigenvectors Q of B are needed: V (U no longer) starts as the identity
    for (int idx = tid; idx < r1 * r1; idx += TH) {
      const int a = idx / r1, b = idx - a * r1;
      sh.V[a * ld + b] = (a == b) ? 1.0 : 0.0;
    }
    __threadfence_block();
    __syncthreads();
    jacobi_for<TH>(sh, sh.V, r1, ld, n);
  } else {
    jacobi_for<TH>(sh, nullptr, r1, ld, n);
  }

  // 4. range filter and trace (fixed order); kidx now flags the eigenvectors kept
  if (tid == 0) {
    const double hi = (1.0 + rho) * g_max;
    double tr = 0.0;
    int r2 = 0;
    for (int j = 0; j < r1; ++j) {
      const double xi = sh.A[j * ld + j];
      const bool in = xi >= 0.0 && xi <= hi;
      sh.kidx[j] = in ? 1 : 0;
      if (in) {
        tr += xi;
        ++r2;
      }
    }
    sh.s[0] = tr;
    if (ranks) {
      ranks[i] = r1;
      ranks[rank_stride + i] = r2;
    }
  }
  __syncthreads();
  double corr = 0.0;
  if (nvh) {  // ||G Q~||_F^2
    double part = 0.0;
    for (int idx = tid; idx < nvh * r1; idx += TH) {
      const int a = idx / r1, j = idx - a * r1;
      if (!sh.kidx[j]) continue;
      double h = 0.0;
      for (int b = 0; b < r1; ++b) h += g[(int64_t)a * r1 + b] * sh.V[j * ld + b];
      part += h * h;
    }
    const double hs = block_sum<TH>(part, sh.red);
    corr = (trw[i] - hs) / nvh;
  }
  if (tid == 0) dos[i] = sh.s[0] + corr;
}

// Backward of Algorithm 4 for one sweep point, truncation sets frozen (the
// estimate is piecewise smooth in K_W, K_Z; the sets change only on a null set).
// In the eigenbasis U of K_W (s = eigenvalues), with F(s) = s^-1/2 on the kept
// set and 0 elsewhere, D = diag(F(s)), Kt = U^T K_Z U, B = D Kt D restricted to
// the kept set, P = projector (embedded in U coordinates) on the eigenvectors of
// B whose eigenvalues pass the range test:
//   phi = tr(P D Kt D),
//   dphi/dK_Z = U (D P D) U^T,
//   dphi/dK_W = U (Gamma o (Kt D P + P D Kt)) U^T      (Daleckii-Krein),
// Gamma_jk = (F(s_j) - F(s_k)) / (s_j - s_k), Gamma_jj = F'(s_j) = -s_j^-3/2 / 2 on
// the kept set; kept/kept entries are -1/(sqrt s_j sqrt s_k (sqrt s_j + sqrt s_k)).
// Both are scaled by phibar[i].  Scratch per point (at scratch + i scr_stride): 3 N_v x N_v
// doubles (U, Kt, and one product), plus the Jacobi matrices above N_v = 96.  With `only`
// set, point i is skipped unless only[i scr_stride] is 1.
template <int TH>
__global__ void __launch_bounds__(TH) geneig_backward_kernel(int nv, const double* __restrict__ k_w,
                                                                     const double* __restrict__ k_z, double g_max,
                                                                     double tau, double rho,
                                                                     const double* __restrict__ phibar,
                                                                     double* __restrict__ kw_bar,
                                                                     double* __restrict__ kz_bar,
                                                                     double* __restrict__ scratch,
                                                                     const double* __restrict__ s_floor,
                                                                     int64_t scr_stride,
                                                                     const double* __restrict__ only) {
  extern __shared__ double lds[];
  const int n = nv;
  const int ld = n + 1;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (only && only[i * scr_stride] != 1.0) return;  // a point the tridiagonal path finished
  const double* kw = k_w + i * nn;
  const double* kz = k_z + i * nn;
  double* ug = scratch + i * scr_stride;  // U
  double* ktg = ug + nn;                                                    // Kt = U^T K_Z U
  double* tg = ug + 2 * nn;                                                 // products
  GeShared sh;
  ge_layout(sh, lds, n, ug + 3 * nn, TH);
  double* f = sh.scale;  // F(s_j) for every j (0 when dropped)
  double* kwb = kw_bar + i * nn;
  double* kzb = kz_bar + i * nn;
  const double pb = phibar[i];

  // 1. eig(K_W)
  for (int idx = tid; idx < n * n; idx += TH) {
    const int r = idx / n, c = idx - r * n;
    sh.A[r * ld + c] = kw[idx];
    sh.V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_for<TH>(sh, sh.V, n, ld, n);
  for (int j = tid; j < n; j += TH) sh.s[j] = sh.A[j * ld + j];
  for (int idx = tid; idx < n * n; idx += TH) ug[idx] = sh.V[(idx % n) * ld + idx / n];
  __syncthreads();
  // 2. truncation (as in the forward kernel)
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, sh.s[j]);
    int r1 = 0;
    const double thr = s_floor ? fmax(tau * smax, s_floor[i]) : tau * smax;
    for (int j = 0; j < n; ++j) {
      const bool keep = smax > 0.0 && sh.s[j] >= thr;
      f[j] = keep ? 1.0 / sqrt(sh.s[j]) : 0.0;
      if (keep) sh.kidx[r1++] = j;
    }
    sh.misc[0] = r1;
  }
  __threadfence_block();
  __syncthreads();
  const int r1 = sh.misc[0];
  if (r1 == 0 || pb == 0.0) {
    for (int idx = tid; idx < n * n; idx += TH) {
      kwb[idx] = 0.0;
      kzb[idx] = 0.0;
    }
    return;
  }
  // 3. Kt = U^T K_Z U: T = K_Z U (global), then Kt = U^T T -> A and global
  for (int idx = tid; idx < n * n; idx += TH) {
    const int r = idx / n, c = idx - r * n;
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += kz[(int64_t)r * n + q] * sh.V[c * ld + q];
    tg[idx] = acc;
  }
  __threadfence_block();
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += TH) {
    const int r = idx / n, c = idx - r * n;
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += sh.V[r * ld + q] * tg[(int64_t)q * n + c];
    sh.A[r * ld + c] = acc;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += TH) {  // symmetrise, keep a copy
    const int r = idx / n, c = idx - r * n;
    ktg[idx] = 0.5 * (sh.A[r * ld + c] + sh.A[c * ld + r]);
  }
  __threadfence_block();
  __syncthreads();
  // 4. B = D Kt D on the kept set -> A (r1 x r1), eigenvectors -> V
  for (int idx = tid; idx < r1 * r1; idx += TH) {
    const int a = idx / r1, b = idx - a * r1;
    const int ka = sh.kidx[a], kb = sh.kidx[b];
    sh.A[a * ld + b] = f[ka] * ktg[(int64_t)ka * n + kb] * f[kb];
    sh.V[a * ld + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_for<TH>(sh, sh.V, r1, ld, n);
  // 5. P (U coordinates, n x n) = sum over in-range xi of x x^T, embedded -> global tg
  const double hi = (1.0 + rho) * g_max;
  for (int idx = tid; idx < n * n; idx += TH) tg[idx] = 0.0;
  __threadfence_block();
  __syncthreads();
  for (int idx = tid; idx < r1 * r1; idx += TH) {
    const int a = idx / r1, b = idx - a * r1;
    double acc = 0.0;
    for (int j = 0; j < r1; ++j) {
      const double xi = sh.A[j * ld + j];
      if (xi >= 0.0 && xi <= hi) acc += sh.V[j * ld + a] * sh.V[j * ld + b];
    }
    tg[(int64_t)sh.kidx[a] * n + sh.kidx[b]] = acc;
  }
  __threadfence_block();
  __syncthreads();
  // 6. M1 = Gamma o (Kt D P + P D Kt) -> V;  M2 = D P D -> A
  for (int idx = tid; idx < n * n; idx += TH) {
    const int j = idx / n, k = idx - j * n;
    double acc = 0.0;  // (Kt D P)[j][k]
    for (int q = 0; q < n; ++q) acc += ktg[(int64_t)j * n + q] * f[q] * tg[(int64_t)q * n + k];
    sh.V[j * ld + k] = acc;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += TH) {
    const int j = idx / n, k = idx - j * n;
    if (j > k) continue;
    const double sj = sh.s[j], sk = sh.s[k];
    const bool kj = f[j] != 0.0, kk = f[k] != 0.0;
    double g;
    if (j == k) {
      g = kj ? -0.5 * f[j] * f[j] * f[j] : 0.0;
    } else if (kj && kk) {
      const double qj = sqrt(sj), qk = sqrt(sk);
      g = -1.0 / (qj * qk * (qj + qk));
    } else if (kj || kk) {
      g = (f[j] - f[k]) / (sj - sk);
    } else {
      g = 0.0;
    }
    const double h = sh.V[j * ld + k] + sh.V[k * ld + j];
    sh.V[j * ld + k] = g * h;
    sh.V[k * ld + j] = g * h;
  }
  for (int idx = tid; idx < n * n; idx += TH) {
    const int j = idx / n, k = idx - j * n;
    sh.A[j * ld + k] = f[j] * tg[idx] * f[k];
  }
  __syncthreads();
  // 7. back to the original coordinates: X = U M U^T, for M1 (-> kw_bar) and M2 (-> kz_bar)
  for (int which = 0; which < 2; ++which) {
    const double* m = which == 0 ? sh.V : sh.A;
    double* out = which == 0 ? kwb : kzb;
    for (int idx = tid; idx < n * n; idx += TH) {  // T = U M
      const int r = idx / n, c = idx - r * n;
      double acc = 0.0;
      for (int q = 0; q < n; ++q) acc += ug[(int64_t)r * n + q] * m[q * ld + c];
      tg[idx] = acc;
    }
    __threadfence_block();
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += TH) {  // out = T U^T
      const int r = idx / n, c = idx - r * n;
      double acc = 0.0;
      for (int q = 0; q < n; ++q) acc += tg[(int64_t)r * n + q] * ug[(int64_t)c * n + q];
      out[idx] = pb * acc;
    }
    __threadfence_block();
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// N_v above 48, the trace without the hybrid term: the two symmetric eigenproblems go through
// a tridiagonal matrix.  (Jacobi there pays for rotating whole N_v x N_v matrices once
// per round; the reduction reads the trailing block once per column instead.)
//   a. geneig_tri_reduce_kernel: Householder reduction Q^T K_W Q = T (T tridiagonal: d
//      on the diagonal, e[i] coupling i and i + 1), the reflectors kept in the rows of
//      the reduced matrix;
//   b. geneig_tri_ql_kernel: implicit QL with Wilkinson shifts on T, one wave per point,
//      its plane rotations recorded in order (Y = their product: T = Y S Y^T);
//   c. geneig_tri_vectors_kernel: U = Q Y row by row, 64 rows per workgroup in LDS, from
//      the reflectors and the record; row j of the transposed array is eigenvector j
//      (the layout of the Jacobi path);
//   d. geneig_tri_trace_kernel: truncation, B, its reduction (as in a), its eigenvalues
//      by bisection on the Sturm counts, one lane per eigenvalue, and the trace.
// A point whose QL runs past its iteration or record limit is redone by the Jacobi
// kernel, which skips the others.
// ---------------------------------------------------------------------------
constexpr int GT_TH = 256;           // one lane per matrix row or column (n <= 256)
constexpr int GT_MAX_QL = 30;        // QL iterations allowed per eigenvalue, on average
constexpr double GT_EPS = 0x1p-52;   // deflation and bisection tolerance unit
constexpr int GT_U = 8;              // loads a lane issues before it uses the first

struct TriShared {
  double d[GE_MAX_NV];
  double e[GE_MAX_NV];
  double tau[GE_MAX_NV];
  double v[2][GE_MAX_NV];  // this step's reflector and the next one's
  double w[2][GE_MAX_NV];  // this step's w and the next step's p
  double s[GE_MAX_NV];
  double scale[GE_MAX_NV];
  double red[GT_TH / 64];
  int kidx[GE_MAX_NV];
  int misc[4];
};

// Sum over the workgroup: a butterfly in each wave (lane 0's value taken), then the
// waves' sums in a fixed order; every lane returns the same value.
__device__ __forceinline__ double gt_sum(double v, double* red) {
  static_assert(GT_TH == 256, "four waves");
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  v = __shfl(v, 0);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// The reflector of x (m entries, global): H = I - tau v v^T with v_0 = 1 maps x to
// beta e_1 (tau = 0, beta = x_0 when x_1.. are all 0).  v goes to vout; returns tau, beta
// in *beta.  Every lane must call it.
__device__ __forceinline__ double gt_reflector(const double* x, int m, double* vout, double* beta, TriShared& sh) {
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int j = 1 + tid; j < m; j += GT_TH) part += x[j] * x[j];
  const double sigma2 = gt_sum(part, sh.red);
  const double alpha = x[0];
  double tau = 0.0, b = alpha, scl = 0.0;
  if (sigma2 > 0.0) {
    const double nrm = sqrt(alpha * alpha + sigma2);
    b = alpha >= 0.0 ? -nrm : nrm;
    tau = (b - alpha) / b;
    scl = 1.0 / (alpha - b);
  }
  for (int j = tid; j < m; j += GT_TH) vout[j] = j == 0 ? 1.0 : x[j] * scl;
  *beta = b;
  return tau;
}

// Householder reduction of the symmetric n x n matrix A (global, row stride ld, both
// triangles held) to T = (d, e).  Step k: x = A[k][k+1..] (= the column below the
// diagonal), H = I - tau v v^T with v_0 = 1 maps x to beta e_1, and the trailing block
// A22 <- H A22 H = A22 - v w^T - w v^T with p = tau A22 v, w = p - (tau/2)(p.v) v.
// Each step after the first reads A22 once: its first row is updated first, the next
// reflector is taken from it, and the pass that updates the rest of A22 also forms the
// next p (the column of A22 below that row is never read again, so it is left as is).
// v is left in A[k][k+1..], tau in sh.tau[k] (0: H = I).
__device__ __forceinline__ void tri_reduce(double* A, int n, int ld, TriShared& sh) {
  const int tid = threadIdx.x;
  if (n >= 3) {  // step 0's reflector and p
    double beta;
    const double tau = gt_reflector(A + 1, n - 1, sh.v[0], &beta, sh);
    if (tid == 0) {
      sh.d[0] = A[0];
      sh.e[0] = beta;
      sh.tau[0] = tau;
    }
    __syncthreads();
    const int m = n - 1;
    const double* a22 = A + ld + 1;
    for (int c = tid; c < m; c += GT_TH) {
      double acc = 0.0;
      int r = 0;
#pragma unroll 1
      for (; r + GT_U <= m; r += GT_U) {
        double a[GT_U];
#pragma unroll
        for (int u = 0; u < GT_U; ++u) a[u] = a22[(int64_t)(r + u) * ld + c];
#pragma unroll
        for (int u = 0; u < GT_U; ++u) acc += a[u] * sh.v[0][r + u];
      }
      for (; r < m; ++r) acc += a22[(int64_t)r * ld + c] * sh.v[0][r];
      sh.w[0][c] = tau * acc;
    }
    __syncthreads();
  }
  for (int k = 0; k + 2 < n; ++k) {
    const int b = k & 1;  // buffers of this step; the next step's are b ^ 1
    const int m = n - k - 1;
    const double tau = sh.tau[k];
    double* vk = sh.v[b];
    double* wk = sh.w[b];
    double* a22 = A + (int64_t)(k + 1) * ld + k + 1;
    if (tau != 0.0) {  // w = p - (tau/2)(p.v) v
      double part = 0.0;
      for (int j = tid; j < m; j += GT_TH) part += wk[j] * vk[j];
      const double h = 0.5 * tau * gt_sum(part, sh.red);
      for (int j = tid; j < m; j += GT_TH) wk[j] -= h * vk[j];
      __syncthreads();
      for (int c = tid; c < m; c += GT_TH) a22[c] -= vk[0] * wk[c] + wk[0] * vk[c];  // row k + 1
      __threadfence_block();
      __syncthreads();
    }
    if (k + 3 < n) {  // next reflector from row k + 1, then the rest of A22 with p'
      double beta;
      const double tau1 = gt_reflector(a22 + 1, m - 1, sh.v[b ^ 1], &beta, sh);
      if (tid == 0) {
        sh.d[k + 1] = a22[0];
        sh.e[k + 1] = beta;
        sh.tau[k + 1] = tau1;
      }
      __syncthreads();
      const double* vn = sh.v[b ^ 1];
      for (int c = 1 + tid; c < m; c += GT_TH) {
        // with tau = 0 (H = I) the column's v_c, w_c are 0 and p was 0, so A22 stays as it is
        const double vc = tau != 0.0 ? vk[c] : 0.0, wc = tau != 0.0 ? wk[c] : 0.0;
        double* col = a22 + c;
        double acc = 0.0;
        int r = 1;
#pragma unroll 1
        for (; r + GT_U <= m; r += GT_U) {
          double a[GT_U];
#pragma unroll
          for (int u = 0; u < GT_U; ++u) a[u] = col[(int64_t)(r + u) * ld];
#pragma unroll
          for (int u = 0; u < GT_U; ++u) {
            const double x = a[u] - (vk[r + u] * wc + wk[r + u] * vc);
            col[(int64_t)(r + u) * ld] = x;
            acc += x * vn[r + u - 1];
          }
        }
        for (; r < m; ++r) {
          const double x = col[(int64_t)r * ld] - (vk[r] * wc + wk[r] * vc);
          col[(int64_t)r * ld] = x;
          acc += x * vn[r - 1];
        }
        sh.w[b ^ 1][c - 1] = tau1 * acc;
      }
    } else if (tau != 0.0) {  // last step: the 2 x 2 block's second row
      for (int c = tid; c < m; c += GT_TH) a22[ld + c] -= vk[1] * wk[c] + wk[1] * vk[c];
    }
    __threadfence_block();
    __syncthreads();
    for (int j = tid; j < m; j += GT_TH) A[(int64_t)k * ld + k + 1 + j] = vk[j];  // row k is no longer read
  }
  __threadfence_block();
  __syncthreads();
  if (tid == 0) {
    if (n >= 2) {
      sh.d[n - 2] = A[(int64_t)(n - 2) * ld + n - 2];
      sh.e[n - 2] = A[(int64_t)(n - 1) * ld + n - 2];
      sh.tau[n - 2] = 0.0;
    }
    sh.d[n - 1] = A[(int64_t)(n - 1) * ld + n - 1];
    sh.e[n - 1] = 0.0;
    sh.tau[n - 1] = 0.0;
  }
  __syncthreads();
}

// Eigenvalue j (ascending) of T = (sh.d, sh.e), n x n, by bisection: the count of
// eigenvalues below x is the number of negative pivots of the LDL^T factorisation of
// T - x I (Sturm), pivots of magnitude <= pivmin replaced by -pivmin.  The search runs
// from the Gershgorin interval until its width is <= 2 eps ||T|| (the midpoint is
// returned).  sh.w[0] must hold e_i^2, and e2max their maximum.
__device__ __forceinline__ double tri_bisect(int j, int n, const TriShared& sh, double glo, double ghi, double e2max) {
  const double tn = fmax(fabs(glo), fabs(ghi));
  const double tol = fmax(2.0 * GT_EPS * tn, 1e-300);
  const double pivmin = 0x1p-1022 * fmax(1.0, e2max);
  double a = glo - tol, b = ghi + tol;
  for (int it = 0; it < 128 && b - a > tol; ++it) {
    const double x = 0.5 * (a + b);
    double q = sh.d[0] - x;
    if (fabs(q) <= pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < n; ++i) {
      q = (sh.d[i] - x) - sh.w[0][i - 1] / q;
      if (fabs(q) <= pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    if (cnt > j)
      b = x;
    else
      a = x;
  }
  return 0.5 * (a + b);
}

// Per-point scratch of the tridiagonal path (row stride n throughout): the matrix being
// reduced (its reflectors, later B) at 0, Z^T at n^2, the QL record (later the n x r1
// product) at 2 n^2, then d, e, tau, the eigenvalues of K_W and the point's status.
struct TriPoint {
  double* a;
  double* zt;
  double* rec;
  double* d;
  double* e;
  double* tau;
  double* eig;
  double* status;  // [0]: 0 when QL finished, 1 when it stopped (the Jacobi kernel redoes the point);
                   // [1]: QL iterations recorded; [2]: rotations recorded
  int* hdr;        // per recorded iteration: m, i0 (its rotations are i = m-1 down to i0)
  __device__ TriPoint(double* base, int n) {
    const int64_t nn = (int64_t)n * n;
    a = base;
    zt = base + nn;
    rec = base + 2 * nn;
    d = base + 6 * nn;
    e = d + n;
    tau = e + n;
    eig = tau + n;
    status = eig + n;
    hdr = (int*)(status + 8);
  }
};
constexpr int GT_REC_NN = 4;   // rotation record capacity, in doubles per n^2
constexpr int GT_REC_IT = 4;   // recorded iterations allowed, per n (about 2 n are taken)

// a. The symmetric part of K_W reduced to tridiagonal form (k_w null: the matrix already in
// the point's scratch).
__global__ void __launch_bounds__(GT_TH) geneig_tri_reduce_kernel(int nv, const double* __restrict__ k_w,
                                                                  double* __restrict__ scratch, int64_t stride) {
  __shared__ TriShared sh;
  const int n = nv;
  const int tid = threadIdx.x;
  const double* kw = k_w ? k_w + blockIdx.x * (int64_t)n * n : nullptr;
  TriPoint pt(scratch + blockIdx.x * stride, n);
  if (k_w) {  // null: the matrix is already in place (the backward's padded B)
    for (int idx = tid; idx < n * n; idx += GT_TH) {
      const int r = idx / n, c = idx - r * n;
      pt.a[idx] = 0.5 * (kw[idx] + kw[(int64_t)c * n + r]);
    }
    __threadfence_block();
    __syncthreads();
  }
  tri_reduce(pt.a, n, n, sh);
  for (int j = tid; j < n; j += GT_TH) {
    pt.d[j] = sh.d[j];
    pt.e[j] = sh.e[j];
    pt.tau[j] = sh.tau[j];
  }
}

// 1/sqrt(x) for normal x > 0: the hardware estimate and two Newton steps
// y <- y (3 - x y^2) / 2 (each at least doubles the correct bits).
__device__ __forceinline__ double gt_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// b. Implicit QL with Wilkinson shifts on T: it finds the next unreduced block [l, m]
// (|e_m| <= eps (|d_m| + |d_m+1|) splits it), takes one shifted iteration on it and
// records the iteration's rotations (c_i, s_i), i = m-1 down to i0, in the stream pt.rec,
// with (m, i0) in pt.hdr.  The rotations are to be applied, in record order, to the
// columns (i, i+1) of Z: z_i+1 <- s z_i + c z_i+1, z_i <- c z_i - s z_i+1.
// Status 1 when the iterations exceed GT_MAX_QL n, or the record its capacity.
// The iteration is one serial chain per point.  Every lane of the wave runs it on the
// same values (each LDS write then stores the same value from every lane), and lane 0
// alone writes the record: with a single lane active, a dependent FP64 chain measured
// 40 cycles per operation with one such wave per point on the GPU, against 13 with the
// wave's 64 lanes active.
__global__ void __launch_bounds__(64) geneig_tri_ql_kernel(int nv, double* __restrict__ scratch, int64_t stride) {
  __shared__ double d[GE_MAX_NV], e[GE_MAX_NV];
  __shared__ double d0[GE_MAX_NV], e0[GE_MAX_NV];  // the block's entries before an iteration
  const int n = nv;
  const bool lead = threadIdx.x == 0;
  TriPoint pt(scratch + blockIdx.x * stride, n);
  for (int j = threadIdx.x; j < n; j += 64) {
    d[j] = pt.d[j];
    e[j] = pt.e[j];
  }
  __syncthreads();
  const int64_t cap = (int64_t)GT_REC_NN * n * n;
  double* rec = pt.rec;
  int64_t pos = 0;
  int l = 0, iters = 0, nrec = 0;
  bool ok = true;
  // first m >= from with |e_m| <= eps (|d_m| + |d_m+1|), n - 1 if none (e_{n-1} = 0): the
  // entries are read GT_U at a time (clamped to the arrays), then tested in order
  auto split_at = [&](int from) {
    for (int m0 = from; m0 < n - 1; m0 += GT_U) {
      double ev[GT_U], dv[GT_U + 1];
#pragma unroll
      for (int u = 0; u < GT_U; ++u) ev[u] = e[min(m0 + u, n - 1)];
#pragma unroll
      for (int u = 0; u <= GT_U; ++u) dv[u] = d[min(m0 + u, n - 1)];
#pragma unroll
      for (int u = 0; u < GT_U; ++u)
        if (m0 + u >= n - 1 || fabs(ev[u]) <= GT_EPS * (fabs(dv[u]) + fabs(dv[u + 1]))) return min(m0 + u, n - 1);
    }
    return n - 1;
  };
  for (;;) {
    int mm = -1;
    while (l < n) {
      const int m = l < n - 1 ? split_at(l) : l;
      if (m == l) {
        ++l;
        continue;
      }
      mm = m;
      break;
    }
    if (mm < 0) break;
    if (++iters > GT_MAX_QL * n || nrec >= GT_REC_IT * n || pos + 2 * (mm - l) > cap) {
      ok = false;
      break;
    }
    // shift: the eigenvalue of the leading 2 x 2 block nearer d_l
    double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
    double r = sqrt(g * g + 1.0);
    const double gs = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
    // The iteration's rotations run without the split test (ss = 0: the block splits at
    // i + 1), which as a branch in the chain cost a fifth of the kernel's time.  A split
    // leaves NaN in the chain from there on, so a NaN g at the end sends the iteration back
    // to the block's entries as they were and through the loop that tests every step.
    for (int j = l + (int)threadIdx.x; j <= mm; j += 64) {
      d0[j] = d[j];
      e0[j] = e[j];
    }
    const int64_t pos0 = pos;
    double s, c, p;
    int i;
    auto iterate = [&](auto tested) {
      constexpr bool TESTED = decltype(tested)::value;
      g = gs;
      s = 1.0;
      c = 1.0;
      p = 0.0;
      pos = pos0;
      i = mm - 1;
      double ei = e[i], di = d[i], di1 = d[i + 1];  // entries the step reads, loaded one step ahead
      for (; i >= l; --i) {
        const double en = e[i > 0 ? i - 1 : 0], dn = d[i > 0 ? i - 1 : 0];  // unconditional loads
        const double f = s * ei, b = c * ei;
        const double ss = f * f + g * g;
        if (TESTED && ss == 0.0) {  // the block splits at i + 1: drop the shift and redo the block
          e[i + 1] = 0.0;
          d[i + 1] = di1 - p;
          e[mm] = 0.0;
          break;
        }
        const double inv = gt_rsqrt(ss);
        r = ss * inv;
        e[i + 1] = r;
        s = f * inv;
        c = g * inv;
        g = di1 - p;
        r = (di - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        if (lead) {
          rec[pos] = c;
          rec[pos + 1] = s;
        }
        pos += 2;
        ei = en;
        di1 = di;
        di = dn;
      }
    };
    iterate(std::false_type{});
    if (__builtin_amdgcn_readfirstlane(g != g ? 1 : 0)) {  // every lane holds the same g
      __syncthreads();
      for (int j = l + (int)threadIdx.x; j <= mm; j += 64) {
        d[j] = d0[j];
        e[j] = e0[j];
      }
      __syncthreads();
      iterate(std::true_type{});
    }
    if (i + 1 < mm) {
      if (lead) {
        pt.hdr[2 * nrec] = mm;
        pt.hdr[2 * nrec + 1] = i + 1;
      }
      ++nrec;
    }
    if (i < l) {
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  for (int j = threadIdx.x; j < n; j += 64) pt.eig[j] = d[j];
  if (lead) {
    pt.status[1] = nrec;
    pt.status[2] = (double)(pos / 2);
    pt.status[0] = ok ? 0.0 : 1.0;
  }
}

// c. Rows of U = Q Y, 64 per workgroup, one per lane (in LDS as L[j][lane], so a wave's
// accesses are contiguous): row r starts as e_r, takes x <- x H_k for k = 0..n-3
// (x - tau (x.v) v^T), then the recorded rotations, and is written to Z^T[.][r].  The
// reflector steps are shared by waves 0..GT_VW-1, each owning the entries j of every row in
// the 8-entry blocks j / 8 = w mod GT_VW: a step's partial products x.v meet in LDS at the
// step's barrier, and each wave then updates its own entries.  The rotations run along a
// row, so wave 0 alone applies them.  Wave GT_VW feeds the others: the reflectors one per
// step through three LDS slots, the rotation record in blocks of GT_BLK through two (an
// iteration may span blocks; wave 0 carries its state across).  Its loads are issued
// GT_VD (GT_RD) steps before their data is due, in rotating register sets, so a step
// waits for none of them; each step ends at a barrier.  The workgroups of one point's row chunks run on one XCD (blockIdx
// modulo 8 picks the XCD), so the record streams from that XCD's L2 after the first.
constexpr int GT_BLK = 512;  // rotations per staged block
constexpr int GT_VD = 3;     // reflector loads in flight
constexpr int GT_RD = 2;     // rotation block loads in flight
constexpr int GT_VW = 3;     // waves sharing the reflector steps (one more feeds them)

__host__ __device__ constexpr size_t tri_vectors_lds_doubles(int n) {
  return (size_t)n * 64 + 2 * GE_MAX_NV + 2 * 2 * GT_BLK + GE_MAX_NV + GT_REC_IT * GE_MAX_NV;
}
__host__ __device__ inline int tri_vectors_groups(int np, int nv) { return (np + 7) / 8 * 8 * ((nv + 63) / 64); }

__global__ void __launch_bounds__(64 * (GT_VW + 1)) geneig_tri_vectors_kernel(int nv, int np,
                                                                              double* __restrict__ scratch,
                                                                              int64_t stride) {
  extern __shared__ double lds[];
  const int n = nv;
  double* L = lds;
  double* vslot = L + n * 64;                  // reflector slots 0 and 1
  double* rslot = vslot + 2 * GE_MAX_NV;       // 2 blocks of rotations
  double* taus = rslot + 2 * 2 * GT_BLK;
  int* hdr = (int*)(taus + GE_MAX_NV);         // 2 GT_REC_IT GE_MAX_NV ints
  // Until the rotation phase, the second rotation block holds reflector slot 2 and the
  // partial products of two steps (GT_VW x 64 each); the feeding wave writes that block
  // only after the barrier that ends the reflector phase.
  double* vslot2 = rslot + 2 * GT_BLK;
  double* part = vslot2 + GE_MAX_NV;
  static_assert(GE_MAX_NV + 2 * GT_VW * 64 <= 2 * GT_BLK, "reflector slot 2 and the partial products");
  auto vref = [&](int k) -> double* {  // reflector k's slot
    const int q = k % 3;
    return q == 2 ? vslot2 : vslot + q * GE_MAX_NV;
  };
  const int nch = (n + 63) / 64;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int point = (slot / nch) * 8 + xcd, ch = slot % nch;
  if (point >= np) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  TriPoint pt(scratch + point * stride, n);
  if (pt.status[0] != 0.0) return;
  const int nit = (int)pt.status[1];
  const int64_t nrot = (int64_t)pt.status[2];
  const int nrefl = n - 2;
  const int r = ch * 64 + lane;
  constexpr int VQ = GE_MAX_NV / 64, RQ = 2 * GT_BLK / 64;

  // Loads are unconditional, at a clamped address inside the point's data; the entries
  // past the end are zeroed when the set is written to LDS.  So the compiler can count the
  // loads in flight and wait for the oldest set only.
  auto load_v = [&](int k, double (&x)[VQ]) {  // reflector k, lane-strided
    const int kk = k < nrefl ? k : nrefl - 1;
    const double* v = pt.a + (int64_t)kk * n + kk + 1;
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
      const int idx = lane + 64 * q;
      x[q] = v[idx < n - kk - 1 ? idx : 0];
    }
  };
  auto put_v = [&](int k, const double (&x)[VQ]) {
    const int m = k < nrefl ? n - k - 1 : 0;
    double* dst = vref(k);
#pragma unroll
    for (int q = 0; q < VQ; ++q) dst[lane + 64 * q] = lane + 64 * q < m ? x[q] : 0.0;
  };
  const int64_t last = 2 * nrot - 1;  // the record's last entry (-1: none)
  auto load_r = [&](int64_t blk, double (&x)[RQ]) {
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int64_t idx = blk * 2 * GT_BLK + lane + 64 * q;
      x[q] = pt.rec[idx <= last ? idx : (last > 0 ? last : 0)];
    }
  };
  auto put_r = [&](int64_t blk, const double (&x)[RQ]) {
    double* dst = rslot + (blk & 1) * 2 * GT_BLK;
#pragma unroll
    for (int q = 0; q < RQ; ++q) dst[lane + 64 * q] = blk * 2 * GT_BLK + lane + 64 * q <= last ? x[q] : 0.0;
  };

  // Step k of the reflector phase on this wave's entries j > k of the row: x.v over them,
  // and x_j <- x_j - y v_j, with v_j at index j - k - 1 of the slot.  Blocks of 8 entries;
  // the block that holds entry k + 1 is cut at it.
  auto refl_first = [&](int k) {  // wave w's first block at or after entry k + 1
    const int b = (k + 1) >> 3;
    return b + (wave - b % GT_VW + GT_VW) % GT_VW;
  };
  auto refl_dot = [&](int k) {
    const double* v = vref(k);
    double acc[4] = {};
    for (int b = refl_first(k); 8 * b < n; b += GT_VW) {
      const int j0 = 8 * b;
      if (j0 > k && j0 + 8 <= n) {
        double xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = L[(j0 + u) * 64 + lane];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u & 3] += xv[u] * v[j0 + u - k - 1];
      } else {
        for (int j = j0 > k ? j0 : k + 1; j < j0 + 8 && j < n; ++j) acc[j & 3] += L[j * 64 + lane] * v[j - k - 1];
      }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
  };
  auto refl_update = [&](int k, double y) {  // reads of a block before its writes
    const double* v = vref(k);
    for (int b = refl_first(k); 8 * b < n; b += GT_VW) {
      const int j0 = 8 * b;
      if (j0 > k && j0 + 8 <= n) {
        double xv[8], vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          xv[u] = L[(j0 + u) * 64 + lane];
          vv[u] = v[j0 + u - k - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) L[(j0 + u) * 64 + lane] = xv[u] - y * vv[u];
      } else {
        for (int j = j0 > k ? j0 : k + 1; j < j0 + 8 && j < n; ++j) L[j * 64 + lane] -= y * v[j - k - 1];
      }
    }
  };

  // every wave passes the same barriers: 1 + nrefl + 1 + nblk
  const int64_t nblk = (nrot + GT_BLK - 1) / GT_BLK;
  if (wave == GT_VW) {
    double vs[GT_VD][VQ];  // reflectors in flight, v_j in set j % GT_VD
    for (int j = lane; j < n; j += 64) taus[j] = pt.tau[j];
    for (int j = lane; j < 2 * nit; j += 64) hdr[j] = pt.hdr[j];
    load_v(0, vs[0]);
    put_v(0, vs[0]);
#pragma unroll
    for (int j = 1; j <= GT_VD; ++j) load_v(j, vs[j % GT_VD]);
    __syncthreads();
    // step k: v_{k+1} (loaded GT_VD steps ago) to LDS, v_{k+1+GT_VD} into the same set
    for (int k0 = 0; k0 < nrefl; k0 += GT_VD) {
#pragma unroll
      for (int u = 0; u < GT_VD; ++u) {
        const int k = k0 + u;
        if (k < nrefl) {
          put_v(k + 1, vs[(u + 1) % GT_VD]);
          load_v(k + 1 + GT_VD, vs[(u + 1) % GT_VD]);
          __syncthreads();
        }
      }
    }
    double rs[GT_RD][RQ];  // rotation blocks in flight, block j in set j % GT_RD
    load_r(0, rs[0]);
    put_r(0, rs[0]);
#pragma unroll
    for (int j = 1; j <= GT_RD; ++j) load_r(j, rs[j % GT_RD]);
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += GT_RD) {
#pragma unroll
      for (int u = 0; u < GT_RD; ++u) {
        const int64_t blk = b0 + u;
        if (blk < nblk) {
          put_r(blk + 1, rs[(u + 1) % GT_RD]);
          load_r(blk + 1 + GT_RD, rs[(u + 1) % GT_RD]);
          __syncthreads();
        }
      }
    }
  } else {
    for (int j = wave; j < n; j += GT_VW) L[j * 64 + lane] = j == r ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < nrefl; ++k) {
      const double tau = taus[k];
      double* pk = part + (k & 1) * GT_VW * 64;
      pk[wave * 64 + lane] = tau != 0.0 ? refl_dot(k) : 0.0;
      __syncthreads();
      if (tau != 0.0) {
        double y = pk[lane];
        for (int w = 1; w < GT_VW; ++w) y += pk[w * 64 + lane];
        refl_update(k, tau * y);
      }
    }
    __syncthreads();
    if (wave != 0) {  // the rotations are wave 0's
      for (int64_t blk = 0; blk < nblk; ++blk) __syncthreads();
    } else {
      int it = 0, t = 0, mm = 0, i0 = 0, cnt = 0;  // the iteration and rotation reached
      double hold = 0.0;
      if (nit > 0) {
        mm = hdr[0];
        i0 = hdr[1];
        cnt = mm - i0;
      }
      for (int64_t blk = 0; blk < nblk; ++blk) {
        const double* rb = rslot + (blk & 1) * 2 * GT_BLK;
        int64_t p = blk * GT_BLK;
        const int64_t pend = p + GT_BLK < nrot ? p + GT_BLK : nrot;
        while (p < pend) {
          if (t == 0) hold = L[mm * 64 + lane];
          const int nh = (int)(cnt - t < pend - p ? cnt - t : pend - p);
          const double* rc = rb + 2 * (p - blk * GT_BLK);
          const int top = mm - 1 - t;  // rotation j of this run is i = top - j
          int j = 0;
          // every LDS read of a batch is issued before its first write: the compiler cannot
          // tell the rows written from the rotations read, so it would not move them
          for (; j + GT_U <= nh; j += GT_U) {
            double z[GT_U], c[GT_U], sn[GT_U];
#pragma unroll
            for (int u = 0; u < GT_U; ++u) {
              z[u] = L[(top - j - u) * 64 + lane];
              c[u] = rc[2 * (j + u)];
              sn[u] = rc[2 * (j + u) + 1];
            }
#pragma unroll
            for (int u = 0; u < GT_U; ++u) {
              L[(top - j - u + 1) * 64 + lane] = sn[u] * z[u] + c[u] * hold;
              hold = c[u] * z[u] - sn[u] * hold;
            }
          }
          for (; j < nh; ++j) {
            const double z = L[(top - j) * 64 + lane];
            const double c = rc[2 * j], sn = rc[2 * j + 1];
            L[(top - j + 1) * 64 + lane] = sn * z + c * hold;
            hold = c * z - sn * hold;
          }
          t += nh;
          p += nh;
          if (t == cnt) {
            L[i0 * 64 + lane] = hold;
            t = 0;
            if (++it < nit) {
              mm = hdr[2 * it];
              i0 = hdr[2 * it + 1];
              cnt = mm - i0;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  if (r < n)
    for (int j = wave; j < n; j += GT_VW + 1) pt.zt[(int64_t)j * n + r] = L[j * 64 + lane];
}

// d. Algorithm 4 steps 2-4 from U, S: truncation, B, its eigenvalues (reduction, then
// bisection) and the trace.
__global__ void __launch_bounds__(GT_TH) geneig_tri_trace_kernel(int nv, const double* __restrict__ k_z,
                                                                 double g_max, double tau, double rho,
                                                                 double* __restrict__ dos,
                                                                 int32_t* __restrict__ ranks, int rank_stride,
                                                                 double* __restrict__ scratch, int64_t stride,
                                                                 const double* __restrict__ s_floor) {
  __shared__ TriShared sh;
  const int n = nv, ld = nv;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const double* kz = k_z + i * (int64_t)n * n;
  TriPoint pt(scratch + i * stride, n);
  if (*pt.status != 0.0) return;  // the Jacobi kernel writes this point
  double* A = pt.a;
  const double* zt = pt.zt;
  double* q = pt.rec;  // the n x r1 product

  // 2. truncation
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, pt.eig[j]);
    int r1 = 0;
    if (smax > 0.0) {
      const double thr = s_floor ? fmax(tau * smax, s_floor[i]) : tau * smax;
      for (int j = 0; j < n; ++j) {
        const double sj = pt.eig[j];
        if (sj >= thr) {
          sh.kidx[r1] = j;
          sh.scale[r1] = 1.0 / sqrt(sj);
          ++r1;
        }
      }
    }
    sh.misc[0] = r1;
  }
  __syncthreads();
  const int r1 = sh.misc[0];
  if (r1 == 0) {
    if (tid == 0) {
      dos[i] = 0.0;
      if (ranks) {
        ranks[i] = 0;
        ranks[rank_stride + i] = 0;
      }
    }
    return;
  }

  // 3a. T = K_Z^T U~ S~^-1/2 (n x r1, row stride r1, in the record's place): lane `row`
  // reads column `row` of K_Z, contiguous across lanes, against GT_U eigenvectors at a
  // time staged in LDS as ub[c][t] (read by all lanes at once).  (K_Z^T in place of K_Z
  // changes B into B^T, which the symmetrisation below takes to the same matrix.)
  __shared__ double ub[GE_MAX_NV * GT_U];
  auto stage_u = [&](int a0) {
    __syncthreads();  // the previous group is no longer read
    for (int idx = tid; idx < GT_U * n; idx += GT_TH) {
      const int t = idx / n, c = idx - t * n;
      ub[c * GT_U + t] = a0 + t < r1 ? zt[(int64_t)sh.kidx[a0 + t] * ld + c] : 0.0;
    }
    __syncthreads();
  };
  for (int a0 = 0; a0 < r1; a0 += GT_U) {
    stage_u(a0);
    if (tid < n) {
      const int row = tid;
      double acc[GT_U] = {};
#pragma unroll 2
      for (int c = 0; c < n; ++c) {
        const double kv = kz[(int64_t)c * n + row];
#pragma unroll
        for (int t = 0; t < GT_U; ++t) acc[t] += kv * ub[c * GT_U + t];
      }
#pragma unroll
      for (int t = 0; t < GT_U; ++t)
        if (a0 + t < r1) q[(int64_t)row * r1 + a0 + t] = acc[t] * sh.scale[a0 + t];
    }
  }
  __threadfence_block();
  __syncthreads();
  // 3b. B = S~^-1/2 U~^T T -> A (r1 x r1, row stride ld): lane b down column b of T
  for (int a0 = 0; a0 < r1; a0 += GT_U) {
    stage_u(a0);
    if (tid < r1) {
      const int b = tid;
      double acc[GT_U] = {};
#pragma unroll 2
      for (int c = 0; c < n; ++c) {
        const double tv = q[(int64_t)c * r1 + b];
#pragma unroll
        for (int t = 0; t < GT_U; ++t) acc[t] += ub[c * GT_U + t] * tv;
      }
#pragma unroll
      for (int t = 0; t < GT_U; ++t)
        if (a0 + t < r1) A[(int64_t)(a0 + t) * ld + b] = acc[t] * sh.scale[a0 + t];
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int idx = tid; idx < r1 * r1; idx += GT_TH) {
    const int a = idx / r1, b = idx - a * r1;
    if (a < b) {
      const double m = 0.5 * (A[(int64_t)a * ld + b] + A[(int64_t)b * ld + a]);
      A[(int64_t)a * ld + b] = m;
      A[(int64_t)b * ld + a] = m;
    }
  }
  __threadfence_block();
  __syncthreads();

  // eig(B): reduction, then bisection
  tri_reduce(A, r1, ld, sh);
  double glo = INFINITY, ghi = -INFINITY, e2max = 0.0;  // every lane: Gershgorin interval
  for (int j = 0; j < r1; ++j) {
    const double rad = (j > 0 ? fabs(sh.e[j - 1]) : 0.0) + (j + 1 < r1 ? fabs(sh.e[j]) : 0.0);
    glo = fmin(glo, sh.d[j] - rad);
    ghi = fmax(ghi, sh.d[j] + rad);
  }
  for (int j = 0; j + 1 < r1; ++j) e2max = fmax(e2max, sh.e[j] * sh.e[j]);
  for (int j = tid; j + 1 < r1; j += GT_TH) sh.w[0][j] = sh.e[j] * sh.e[j];
  __syncthreads();
  for (int j = tid; j < r1; j += GT_TH) sh.s[j] = tri_bisect(j, r1, sh, glo, ghi, e2max);
  __syncthreads();

  // 4. range filter and trace, ascending order
  if (tid == 0) {
    const double hi = (1.0 + rho) * g_max;
    double tr = 0.0;
    int r2 = 0;
    for (int j = 0; j < r1; ++j) {
      const double xi = sh.s[j];
      if (xi >= 0.0 && xi <= hi) {
        tr += xi;
        ++r2;
      }
    }
    dos[i] = tr;
    if (ranks) {
      ranks[i] = r1;
      ranks[rank_stride + i] = r2;
    }
  }
}


// ---------------------------------------------------------------------------
// Backward of Algorithm 4 on the tridiagonal path (N_v > 48), per group of points:
//   a-c on K_W as in the forward path (U, S);
//   geneig_tri_bwd_form_kernel: truncation (F(s) = s^-1/2 kept, 0 dropped), U saved,
//     Kt = U^T K_Z U, and B = D Kt D on the kept set, padded to N_v x N_v with -1 on the
//     padding's diagonal (outside [0, (1 + rho) g_max], so those eigenpairs never enter
//     the projector; the padding stays a separate block through the reduction);
//   a-c on the padded B (reduced in place): its eigenvalues xi and eigenvectors Q;
//   geneig_tri_bwd_finish_kernel: P = sum over in-range xi of q q^T (U coordinates),
//     M1 = Gamma o (Kt D P + P D Kt), M2 = D P D, and kw_bar, kz_bar = phibar U M U^T
//     (the formulas of geneig_backward_kernel).
// A point whose QL stops in either run is redone by geneig_backward_kernel.
// Per-point scratch: the forward path's, then U^T, Kt, F(s), s, the kept indices and
// the point's state (0: on the path, 1: to be redone, 2: done).
// ---------------------------------------------------------------------------
struct TriBwd {
  double* ut;   // U^T: row j = eigenvector j of K_W
  double* kt;   // Kt
  double* f;    // F(s_j)
  double* s;    // s_j
  int* kidx;    // kept indices, r1 of them
  double* state;
  double* r1;
  __device__ TriBwd(double* base, int n) {
    const int64_t nn = (int64_t)n * n;
    ut = base + geneig_tri_point_doubles(n);
    kt = ut + nn;
    f = kt + nn;
    s = f + n;
    kidx = (int*)(s + n);
    state = s + 2 * n;
    r1 = state + 1;
  }
};

// R(r, c) = sum_q X(r, q) Y[q][c] for r < rows, c < cols (<= GT_TH), q < kdim: lane c down
// column c of Y (row-major, contiguous across lanes) against GT_U rows of X at a time,
// staged in LDS as ub[q][t] and read there by every lane at once.  x_at(r, q) gives X;
// X_T says X(r, q) sits at q * ld + r (staged with r fastest) rather than r * ld + q.
template <bool X_T, typename XF, typename OUT>
__device__ __forceinline__ void gt_gemm(int rows, int cols, int kdim, XF x_at, const double* Y, int64_t ldy,
                                        double* ub, OUT out) {
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < rows; r0 += GT_U) {
    __syncthreads();  // the previous group is no longer read
    for (int idx = tid; idx < GT_U * kdim; idx += GT_TH) {
      int t, q;
      if (X_T) {
        t = idx % GT_U;
        q = idx / GT_U;
      } else {
        t = idx / kdim;
        q = idx - t * kdim;
      }
      ub[q * GT_U + t] = r0 + t < rows ? x_at(r0 + t, q) : 0.0;
    }
    __syncthreads();
    if (tid < cols) {
      double acc[GT_U] = {};
#pragma unroll 2
      for (int q = 0; q < kdim; ++q) {
        const double y = Y[(int64_t)q * ldy + tid];
#pragma unroll
        for (int t = 0; t < GT_U; ++t) acc[t] += ub[q * GT_U + t] * y;
      }
#pragma unroll
      for (int t = 0; t < GT_U; ++t)
        if (r0 + t < rows) out(r0 + t, tid, acc[t]);
    }
  }
  __threadfence_block();
  __syncthreads();
}

__global__ void __launch_bounds__(GT_TH) geneig_tri_bwd_form_kernel(int nv, const double* __restrict__ k_z,
                                                                    double tau, const double* __restrict__ phibar,
                                                                    double* __restrict__ kw_bar,
                                                                    double* __restrict__ kz_bar,
                                                                    double* __restrict__ scratch, int64_t stride,
                                                                    const double* __restrict__ s_floor) {
  __shared__ double ub[GE_MAX_NV * GT_U];
  __shared__ int misc[2];
  const int n = nv;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  const double* kz = k_z + i * nn;
  TriPoint pt(scratch + i * stride, n);
  TriBwd bw(scratch + i * stride, n);
  if (pt.status[0] != 0.0) {  // QL on K_W stopped
    if (tid == 0) *bw.state = 1.0;
    return;
  }
  // truncation, as in the forward path
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, pt.eig[j]);
    const double thr = s_floor ? fmax(tau * smax, s_floor[i]) : tau * smax;
    int r1 = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = pt.eig[j];
      const bool keep = smax > 0.0 && sj >= thr;
      bw.s[j] = sj;
      bw.f[j] = keep ? 1.0 / sqrt(sj) : 0.0;
      if (keep) bw.kidx[r1++] = j;
    }
    *bw.r1 = r1;
    misc[0] = r1;
  }
  __syncthreads();
  const int r1 = misc[0];
  if (r1 == 0 || phibar[i] == 0.0) {
    for (int idx = tid; idx < n * n; idx += GT_TH) {
      kw_bar[i * nn + idx] = 0.0;
      kz_bar[i * nn + idx] = 0.0;
    }
    if (tid == 0) *bw.state = 2.0;
    return;
  }
  if (tid == 0) *bw.state = 0.0;
  for (int idx = tid; idx < n * n; idx += GT_TH) bw.ut[idx] = pt.zt[idx];
  __threadfence_block();
  __syncthreads();
  // S1^T = (U^T K_Z)^T into the record's place: S1[b][q] = sum_p U[p][b] K_Z[p][q]
  double* s1t = pt.rec;
  gt_gemm<false>(
      n, n, n, [&](int b, int p) { return bw.ut[(int64_t)b * n + p]; }, kz, n, ub,
      [&](int b, int q, double v) { s1t[(int64_t)q * n + b] = v; });
  // Kt^T[b][a] = sum_r U[r][b] S1[a][r]; stored as it comes (symmetrised next)
  gt_gemm<false>(
      n, n, n, [&](int b, int r) { return bw.ut[(int64_t)b * n + r]; }, s1t, n, ub,
      [&](int b, int a, double v) { bw.kt[(int64_t)b * n + a] = v; });
  for (int idx = tid; idx < n * n; idx += GT_TH) {
    const int a = idx / n, b = idx - a * n;
    if (a < b) {
      const double m = 0.5 * (bw.kt[(int64_t)a * n + b] + bw.kt[(int64_t)b * n + a]);
      bw.kt[(int64_t)a * n + b] = m;
      bw.kt[(int64_t)b * n + a] = m;
    }
  }
  __threadfence_block();
  __syncthreads();
  // the padded B into the reduction's place
  for (int idx = tid; idx < n * n; idx += GT_TH) {
    const int a = idx / n, b = idx - a * n;
    double v;
    if (a < r1 && b < r1) {
      const int ka = bw.kidx[a], kb = bw.kidx[b];
      v = bw.f[ka] * bw.kt[(int64_t)ka * n + kb] * bw.f[kb];
    } else {
      v = a == b ? -1.0 : 0.0;
    }
    pt.a[idx] = v;
  }
}

__global__ void __launch_bounds__(GT_TH) geneig_tri_bwd_finish_kernel(int nv, double g_max, double rho,
                                                                      const double* __restrict__ phibar,
                                                                      double* __restrict__ kw_bar,
                                                                      double* __restrict__ kz_bar,
                                                                      double* __restrict__ scratch, int64_t stride) {
  __shared__ double ub[GE_MAX_NV * GT_U];
  const int n = nv;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  TriPoint pt(scratch + i * stride, n);
  TriBwd bw(scratch + i * stride, n);
  if (*bw.state != 0.0) return;  // redone by Jacobi, or done
  if (pt.status[0] != 0.0) {     // QL on B stopped
    if (tid == 0) *bw.state = 1.0;
    return;
  }
  const int r1 = (int)*bw.r1;
  const double hi = (1.0 + rho) * g_max;
  const double pb = phibar[i];
  double* kwb = kw_bar + i * nn;
  double* kzb = kz_bar + i * nn;
  const double* q = pt.zt;   // eigenvector j of B in row j (entries a < r1)
  double* pu = pt.rec;       // P in U coordinates
  double* m1 = pt.a;         // Kt D P, then M1
  double* tt = pt.zt;        // M U^T once Q is spent
  for (int idx = tid; idx < n * n; idx += GT_TH) pu[idx] = 0.0;
  __threadfence_block();
  __syncthreads();
  // P[ka][kb] = sum over in-range j of q_j[a] q_j[b], a, b < r1
  gt_gemm<true>(
      r1, r1, n,
      [&](int a, int j) {
        const double xi = pt.eig[j];
        return xi >= 0.0 && xi <= hi ? q[(int64_t)j * n + a] : 0.0;
      },
      q, n, ub, [&](int a, int b, double v) { pu[(int64_t)bw.kidx[a] * n + bw.kidx[b]] = v; });
  // Kt D P
  gt_gemm<false>(
      n, n, n, [&](int j, int c) { return bw.kt[(int64_t)j * n + c] * bw.f[c]; }, pu, n, ub,
      [&](int j, int k, double v) { m1[(int64_t)j * n + k] = v; });
  // M1 = Gamma o (X + X^T), Gamma the divided differences of F
  for (int idx = tid; idx < n * n; idx += GT_TH) {
    const int j = idx / n, k = idx - j * n;
    if (j > k) continue;
    const double sj = bw.s[j], sk = bw.s[k], fj = bw.f[j], fk = bw.f[k];
    const bool kj = fj != 0.0, kk = fk != 0.0;
    double g;
    if (j == k) {
      g = kj ? -0.5 * fj * fj * fj : 0.0;
    } else if (kj && kk) {
      const double qj = sqrt(sj), qk = sqrt(sk);
      g = -1.0 / (qj * qk * (qj + qk));
    } else if (kj || kk) {
      g = (fj - fk) / (sj - sk);
    } else {
      g = 0.0;
    }
    const double h = m1[(int64_t)j * n + k] + m1[(int64_t)k * n + j];
    m1[(int64_t)j * n + k] = g * h;
    m1[(int64_t)k * n + j] = g * h;
  }
  __threadfence_block();
  __syncthreads();
  // kw_bar = phibar U M1 U^T: (M1 U^T)[q][r] = sum_c M1[q][c] U[r][c], then U (M1 U^T)
  gt_gemm<false>(
      n, n, n, [&](int r, int c) { return m1[(int64_t)r * n + c]; }, bw.ut, n, ub,
      [&](int r, int c, double v) { tt[(int64_t)r * n + c] = v; });
  gt_gemm<true>(
      n, n, n, [&](int r, int c) { return bw.ut[(int64_t)c * n + r]; }, tt, n, ub,
      [&](int r, int c, double v) { kwb[(int64_t)r * n + c] = pb * v; });
  // kz_bar = phibar U M2 U^T, M2 = D P D
  gt_gemm<false>(
      n, n, n, [&](int r, int c) { return bw.f[r] * pu[(int64_t)r * n + c] * bw.f[c]; }, bw.ut, n, ub,
      [&](int r, int c, double v) { tt[(int64_t)r * n + c] = v; });
  gt_gemm<true>(
      n, n, n, [&](int r, int c) { return bw.ut[(int64_t)c * n + r]; }, tt, n, ub,
      [&](int r, int c, double v) { kzb[(int64_t)r * n + c] = pb * v; });
}


// ---------------------------------------------------------------------------
// The trace with RESS-DGC's hybrid term (Algorithm 6, N~_v = nvh columns of W~), N_v > 48:
//   a-c on K_W (U, S);
//   geneig_tri_hyb_form_kernel: truncation, U~ = U~ S~^-1/2 (N_v x r1), G^T = (K_C U~)^T,
//     B = U~^T K_Z U~ padded to N_v x N_v with -1 on the padding's diagonal;
//   a-c on the padded B (its eigenvalues xi, eigenvectors Q);
//   geneig_tri_hyb_finish_kernel: the trace of the in-range xi and the correction
//     (Tr K_W~ - ||G Q~||_F^2) / N~_v, Q~ the in-range eigenvectors (the padding's
//     eigenvalues, -1, are never in range).
// status[3] of a point holds r1, status[4] its state (0: on the path, 1: redone by
// Jacobi, 2: done); U~ and K_Z U~ go through the record's place, G^T through hscr.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(GT_TH) geneig_tri_hyb_form_kernel(int nv, int nvh, const double* __restrict__ k_z,
                                                                    const double* __restrict__ k_c, double tau,
                                                                    const double* __restrict__ trw,
                                                                    double* __restrict__ dos,
                                                                    int32_t* __restrict__ ranks, int rank_stride,
                                                                    double* __restrict__ scratch, int64_t stride,
                                                                    double* __restrict__ hscr,
                                                                    const double* __restrict__ s_floor) {
  __shared__ double ub[GE_MAX_NV * GT_U];
  __shared__ double scale[GE_MAX_NV];
  __shared__ int kidx[GE_MAX_NV];
  __shared__ int misc[1];
  const int n = nv;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  const double* kz = k_z + i * nn;
  const double* kc = k_c + (int64_t)i * nvh * n;
  double* gt = hscr + (int64_t)i * nvh * n;
  TriPoint pt(scratch + i * stride, n);
  if (pt.status[0] != 0.0) {  // QL on K_W stopped
    if (tid == 0) pt.status[4] = 1.0;
    return;
  }
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, pt.eig[j]);
    int r1 = 0;
    if (smax > 0.0) {
      const double thr = s_floor ? fmax(tau * smax, s_floor[i]) : tau * smax;
      for (int j = 0; j < n; ++j)
        if (pt.eig[j] >= thr) {
          kidx[r1] = j;
          scale[r1] = 1.0 / sqrt(pt.eig[j]);
          ++r1;
        }
    }
    misc[0] = r1;
    pt.status[3] = r1;
    pt.status[4] = r1 == 0 ? 2.0 : 0.0;
    if (r1 == 0) {  // C~ is empty: only Tr K_W~ / N~_v remains
      dos[i] = trw[i] / nvh;
      if (ranks) {
        ranks[i] = 0;
        ranks[rank_stride + i] = 0;
      }
    }
  }
  __syncthreads();
  const int r1 = misc[0];
  if (r1 == 0) return;
  double* ut = pt.rec;                   // U~ S~^-1/2, N_v x r1
  double* tz = pt.rec + (int64_t)n * r1;  // K_Z^T U~ S~^-1/2, N_v x r1
  for (int idx = tid; idx < n * r1; idx += GT_TH) {
    const int c = idx / r1, b = idx - c * r1;
    ut[idx] = pt.zt[(int64_t)kidx[b] * n + c] * scale[b];
  }
  __threadfence_block();
  __syncthreads();
  // G^T[b][a] = sum_c K_C[a][c] U~[c][b]
  gt_gemm<false>(
      nvh, r1, n, [&](int a, int c) { return kc[(int64_t)a * n + c]; }, ut, r1, ub,
      [&](int a, int b, double v) { gt[(int64_t)b * nvh + a] = v; });
  // K_Z^T U~ (K_Z^T for K_Z: B becomes B^T, which the symmetrisation takes to the same matrix)
  gt_gemm<true>(
      n, r1, n, [&](int r, int c) { return kz[(int64_t)c * n + r]; }, ut, r1, ub,
      [&](int r, int b, double v) { tz[(int64_t)r * r1 + b] = v; });
  // B = U~^T (K_Z^T U~) into the reduction's place
  gt_gemm<true>(
      r1, r1, n, [&](int a, int c) { return ut[(int64_t)c * r1 + a]; }, tz, r1, ub,
      [&](int a, int b, double v) { pt.a[(int64_t)a * n + b] = v; });
  for (int idx = tid; idx < n * n; idx += GT_TH) {
    const int a = idx / n, b = idx - a * n;
    if (a < r1 && b < r1) {
      if (a < b) {
        const double m = 0.5 * (pt.a[(int64_t)a * n + b] + pt.a[(int64_t)b * n + a]);
        pt.a[(int64_t)a * n + b] = m;
        pt.a[(int64_t)b * n + a] = m;
      }
    } else {
      pt.a[idx] = a == b ? -1.0 : 0.0;
    }
  }
}

__global__ void __launch_bounds__(GT_TH) geneig_tri_hyb_finish_kernel(int nv, int nvh, double g_max, double rho,
                                                                      const double* __restrict__ trw,
                                                                      double* __restrict__ dos,
                                                                      int32_t* __restrict__ ranks, int rank_stride,
                                                                      double* __restrict__ scratch, int64_t stride,
                                                                      const double* __restrict__ hscr) {
  __shared__ double ub[GE_MAX_NV * GT_U];
  __shared__ double red[GT_TH / 64];
  const int n = nv;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  TriPoint pt(scratch + i * stride, n);
  if (pt.status[4] != 0.0) return;  // redone by Jacobi, or done
  if (pt.status[0] != 0.0) {        // QL on B stopped
    if (tid == 0) pt.status[4] = 1.0;
    return;
  }
  const int r1 = (int)pt.status[3];
  const double hi = (1.0 + rho) * g_max;
  const double* gt = hscr + (int64_t)i * nvh * n;
  // ||G Q~||_F^2: row j of H^T = Q~^T G^T is sum_b q_j[b] G^T[b][.], lane a summing squares
  double part = 0.0;
  gt_gemm<false>(
      n, nvh, r1,
      [&](int j, int b) {
        const double xi = pt.eig[j];
        return xi >= 0.0 && xi <= hi ? pt.zt[(int64_t)j * n + b] : 0.0;
      },
      gt, nvh, ub, [&](int, int, double v) { part += v * v; });
  const double hs = gt_sum(part, red);
  if (tid == 0) {
    double tr = 0.0;
    int r2 = 0;
    for (int j = 0; j < n; ++j) {
      const double xi = pt.eig[j];
      if (xi >= 0.0 && xi <= hi) {
        tr += xi;
        ++r2;
      }
    }
    dos[i] = tr + (trw[i] - hs) / nvh;
    if (ranks) {
      ranks[i] = r1;
      ranks[rank_stride + i] = r2;
    }
  }
}

}  // namespace

// Threads per point: the Jacobi rounds are latency-bound at one workgroup per CU, so the
// larger matrices take more waves (measured on the benchmark's pencils: N_v = 80 runs in
// 0.63x the time with 512 threads; N_v = 40 is fastest with 256).
int geneig_threads(int nv) { return nv <= 48 ? 256 : nv <= GE_LDS_NV ? 512 : GE_MAX_THREADS; }

size_t geneig_lds_bytes(int nv) {
  const size_t n = (size_t)nv, ld = n + 1;
  const size_t mats = (size_t)geneig_lds_matrices(nv) * n * ld;
  return (mats + 2 * GE_MAX_NV + GE_MAX_NV + (size_t)geneig_threads(nv)) * sizeof(double) +
         (GE_MAX_NV + GE_MAX_NV + 4) * sizeof(int);
}

template <int TH>
hipError_t launch_backward_t(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                             double rho, const double* phibar, double* kw_bar, double* kz_bar, double* scratch,
                             const double* s_floor, size_t lds, hipStream_t stream, int64_t scr_stride,
                             const double* only) {
  hipError_t err = hipFuncSetAttribute((const void*)geneig_backward_kernel<TH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(geneig_backward_kernel<TH>, dim3(ntb), dim3(TH), lds, stream, nv, k_w, k_z, g_max, tau, rho,
                     phibar, kw_bar, kz_bar, scratch, s_floor, scr_stride, only);
  return hipGetLastError();
}

hipError_t launch_jacobi_backward(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                                  double rho, const double* phibar, double* kw_bar, double* kz_bar, double* scratch,
                                  const double* s_floor, hipStream_t stream, int64_t scr_stride, const double* only) {
  const size_t lds = geneig_lds_bytes(nv);
  switch (geneig_threads(nv)) {
    case 256:
      return launch_backward_t<256>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch, s_floor, lds,
                                    stream, scr_stride, only);
    case 512:
      return launch_backward_t<512>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch, s_floor, lds,
                                    stream, scr_stride, only);
    default:
      return launch_backward_t<GE_MAX_THREADS>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch,
                                               s_floor, lds, stream, scr_stride, only);
  }
}

template <int TH>
hipError_t launch_trace_t(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                          double rho, double* dos, int32_t* ranks, double* scratch, int nvh, const double* k_c,
                          const double* trw, double* hscr, const double* s_floor, int rank_stride, size_t lds,
                          hipStream_t stream, int64_t scr_stride, const double* only) {
  hipError_t err = hipFuncSetAttribute((const void*)geneig_trace_kernel<TH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(geneig_trace_kernel<TH>, dim3(ntb), dim3(TH), lds, stream, nv, k_w, k_z, g_max, tau, rho, dos,
                     ranks, rank_stride, scratch, nvh, k_c, trw, hscr, s_floor, scr_stride, only);
  return hipGetLastError();
}

// The Jacobi kernel for the threads N_v takes.
hipError_t launch_jacobi_trace(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                               double rho, double* dos, int32_t* ranks, double* scratch, int nvh, const double* k_c,
                               const double* trw, double* hscr, const double* s_floor, int rank_stride,
                               hipStream_t stream, int64_t scr_stride, const double* only) {
  const size_t lds = geneig_lds_bytes(nv);
  switch (geneig_threads(nv)) {
    case 256:
      return launch_trace_t<256>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw, hscr,
                                 s_floor, rank_stride, lds, stream, scr_stride, only);
    case 512:
      return launch_trace_t<512>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw, hscr,
                                 s_floor, rank_stride, lds, stream, scr_stride, only);
    default:
      return launch_trace_t<GE_MAX_THREADS>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw,
                                            hscr, s_floor, rank_stride, lds, stream, scr_stride, only);
  }
}

hipError_t launch_geneig_backward(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                                  double rho, const double* phibar, double* kw_bar, double* kz_bar, double* scratch,
                                  hipStream_t stream, const double* s_floor) {
  if (nv < 1 || nv > GE_MAX_NV) return hipErrorInvalidValue;
  if (!geneig_tri_path(nv))
    return launch_jacobi_backward(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch, s_floor,
                                  stream, geneig_backward_scratch_doubles(nv), nullptr);
  // the tridiagonal path on K_W, then on the padded B, kGeTriChunk points at a time
  const int64_t stride = geneig_tri_bwd_point_doubles(nv);
  const int64_t nn = (int64_t)nv * nv;
  const int64_t state_off = geneig_tri_point_doubles(nv) + 2 * nn + 3 * (int64_t)nv;  // TriBwd::state
  const size_t vec_lds = tri_vectors_lds_doubles(nv) * sizeof(double);
  hipError_t err = hipFuncSetAttribute((const void*)geneig_tri_vectors_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)vec_lds);
  if (err != hipSuccess) return err;
  for (int i0 = 0; i0 < ntb; i0 += kGeTriChunk) {
    const int np = std::min(kGeTriChunk, ntb - i0);
    const double* kw = k_w + i0 * nn;
    const double* kz = k_z + i0 * nn;
    const double* pb = phibar + i0;
    double* kwb = kw_bar + i0 * nn;
    double* kzb = kz_bar + i0 * nn;
    const double* sf = s_floor ? s_floor + i0 : nullptr;
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(geneig_tri_reduce_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, pass ? nullptr : kw,
                         scratch, stride);
      hipLaunchKernelGGL(geneig_tri_ql_kernel, dim3(np), dim3(64), 0, stream, nv, scratch, stride);
      hipLaunchKernelGGL(geneig_tri_vectors_kernel, dim3(tri_vectors_groups(np, nv)), dim3(64 * (GT_VW + 1)), vec_lds, stream,
                         nv, np, scratch, stride);
      if (pass == 0)
        hipLaunchKernelGGL(geneig_tri_bwd_form_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, kz, tau, pb, kwb, kzb,
                           scratch, stride, sf);
      else
        hipLaunchKernelGGL(geneig_tri_bwd_finish_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, g_max, rho, pb, kwb,
                           kzb, scratch, stride);
    }
    err = launch_jacobi_backward(nv, np, kw, kz, g_max, tau, rho, pb, kwb, kzb, scratch, sf, stream, stride,
                                 scratch + state_off);
    if (err != hipSuccess) return err;
  }
  return hipGetLastError();
}

hipError_t launch_geneig_trace(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                               double rho, double* dos, int32_t* ranks, double* scratch, hipStream_t stream,
                               int nvh, const double* k_c, const double* trw, double* hscr,
                               const double* s_floor, int rank_stride) {
  if (nv < 1 || nv > GE_MAX_NV) return hipErrorInvalidValue;
  if (nvh < 0 || (nvh > 0 && (!k_c || !trw || !hscr))) return hipErrorInvalidValue;
  if (rank_stride <= 0) rank_stride = ntb;
  if (!geneig_tri_path(nv))
    return launch_jacobi_trace(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw, hscr, s_floor,
                               rank_stride, stream, geneig_scratch_doubles(nv), nullptr);
  // the tridiagonal path, kGeTriChunk points at a time through the same scratch
  const int64_t stride = geneig_tri_point_doubles(nv);
  const int64_t nn = (int64_t)nv * nv;
  const size_t vec_lds = tri_vectors_lds_doubles(nv) * sizeof(double);
  hipError_t err = hipFuncSetAttribute((const void*)geneig_tri_vectors_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)vec_lds);
  if (err != hipSuccess) return err;
  for (int i0 = 0; i0 < ntb; i0 += kGeTriChunk) {
    const int np = std::min(kGeTriChunk, ntb - i0);
    const double* kw = k_w + i0 * nn;
    const double* kz = k_z + i0 * nn;
    int32_t* rk = ranks ? ranks + i0 : nullptr;
    const double* sf = s_floor ? s_floor + i0 : nullptr;
    hipLaunchKernelGGL(geneig_tri_reduce_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, kw, scratch, stride);
    hipLaunchKernelGGL(geneig_tri_ql_kernel, dim3(np), dim3(64), 0, stream, nv, scratch, stride);
    hipLaunchKernelGGL(geneig_tri_vectors_kernel, dim3(tri_vectors_groups(np, nv)), dim3(64 * (GT_VW + 1)), vec_lds, stream, nv,
                       np, scratch, stride);
    if (nvh == 0) {
      hipLaunchKernelGGL(geneig_tri_trace_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, kz, g_max, tau, rho,
                         dos + i0, rk, rank_stride, scratch, stride, sf);
      err = launch_jacobi_trace(nv, np, kw, kz, g_max, tau, rho, dos + i0, rk, scratch, 0, nullptr, nullptr, nullptr,
                                sf, rank_stride, stream, stride, scratch + 6 * nn + 4 * nv);
    } else {  // B through the same kernels, then the trace and the hybrid term
      const double* kc = k_c + (int64_t)i0 * nvh * nv;
      double* hs = hscr + (int64_t)i0 * nvh * nv;
      hipLaunchKernelGGL(geneig_tri_hyb_form_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, nvh, kz, kc, tau,
                         trw + i0, dos + i0, rk, rank_stride, scratch, stride, hs, sf);
      hipLaunchKernelGGL(geneig_tri_reduce_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, (const double*)nullptr,
                         scratch, stride);
      hipLaunchKernelGGL(geneig_tri_ql_kernel, dim3(np), dim3(64), 0, stream, nv, scratch, stride);
      hipLaunchKernelGGL(geneig_tri_vectors_kernel, dim3(tri_vectors_groups(np, nv)), dim3(64 * (GT_VW + 1)), vec_lds, stream,
                         nv, np, scratch, stride);
      hipLaunchKernelGGL(geneig_tri_hyb_finish_kernel, dim3(np), dim3(GT_TH), 0, stream, nv, nvh, g_max, rho,
                         trw + i0, dos + i0, rk, rank_stride, scratch, stride, hs);
      err = launch_jacobi_trace(nv, np, kw, kz, g_max, tau, rho, dos + i0, rk, scratch, nvh, kc, trw + i0, hs, sf,
                                rank_stride, stream, stride, scratch + 6 * nn + 4 * nv + 4);
    }
    if (err != hipSuccess) return err;
  }
  return hipGetLastError();
}

}  // namespace ssm
