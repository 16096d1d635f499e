// Algorithm 4 (truncated generalised eigenvalue problem) and the trace of
// Algorithm 5 (step 13), one workgroup per sweep point, in FP64:
//
//   1. W^T Z = U S U^T                     (cyclic Jacobi, eigenvectors kept)
//   2. keep s_j >= tau max_i s_i            (nothing kept, trace 0, if max s <= 0)
//   3. B = S~^-1/2 U~^T (Z^T Z) U~ S~^-1/2,  eig(B) = xi   (Jacobi, values only)
//   4. keep xi in [0, (1 + rho) g_max], g_max = 1/(N sqrt(2 pi sigma^2))
//   trace = sum of kept xi, r1 = |kept s|, r2 = |kept xi|.
//
// Jacobi: parallel cyclic sweeps in round-robin (tournament) order, so each round
// rotates N_v/2 disjoint index pairs at once: the pair angles are computed first
// (Golub & Van Loan, symmetric 2x2 Schur), then the rows of every pair are rotated,
// then the columns (and the eigenvector columns).  The pivot entries are set to
// exactly zero.  A sweep starts only while off(A)_F > 1e-14 ||A||_F.
// The matrix and its eigenvectors live in LDS for N_v <= 96 (2 * 96 * 97 doubles), the
// matrix alone up to N_v = 128 (eigenvectors in the point's global scratch), both in
// global scratch above that (N_v <= 256); the N_v x r1 product
// Z^T Z U~ S~^-1/2 goes through the same per-point scratch.
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
                                                                  const double* __restrict__ s_floor) {
  extern __shared__ double lds[];
  const int n = nv;
  const int ld = n + 1;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  const double* kw = k_w + i * nn;
  const double* kz = k_z + i * nn;
  double* tmat = scratch + i * (int64_t)geneig_scratch_doubles(nv);
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
// Both are scaled by phibar[i].  Scratch per point: 3 N_v x N_v doubles
// (U, Kt, and one product).
template <int TH>
__global__ void __launch_bounds__(TH) geneig_backward_kernel(int nv, const double* __restrict__ k_w,
                                                                     const double* __restrict__ k_z, double g_max,
                                                                     double tau, double rho,
                                                                     const double* __restrict__ phibar,
                                                                     double* __restrict__ kw_bar,
                                                                     double* __restrict__ kz_bar,
                                                                     double* __restrict__ scratch,
                                                                     const double* __restrict__ s_floor) {
  extern __shared__ double lds[];
  const int n = nv;
  const int ld = n + 1;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  const double* kw = k_w + i * nn;
  const double* kz = k_z + i * nn;
  double* ug = scratch + i * (int64_t)geneig_backward_scratch_doubles(nv);  // U
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
                             const double* s_floor, size_t lds, hipStream_t stream) {
  hipError_t err = hipFuncSetAttribute((const void*)geneig_backward_kernel<TH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(geneig_backward_kernel<TH>, dim3(ntb), dim3(TH), lds, stream, nv, k_w, k_z, g_max, tau, rho,
                     phibar, kw_bar, kz_bar, scratch, s_floor);
  return hipGetLastError();
}

template <int TH>
hipError_t launch_trace_t(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                          double rho, double* dos, int32_t* ranks, double* scratch, int nvh, const double* k_c,
                          const double* trw, double* hscr, const double* s_floor, int rank_stride, size_t lds,
                          hipStream_t stream) {
  hipError_t err = hipFuncSetAttribute((const void*)geneig_trace_kernel<TH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(geneig_trace_kernel<TH>, dim3(ntb), dim3(TH), lds, stream, nv, k_w, k_z, g_max, tau, rho, dos,
                     ranks, rank_stride, scratch, nvh, k_c, trw, hscr, s_floor);
  return hipGetLastError();
}

hipError_t launch_geneig_backward(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                                  double rho, const double* phibar, double* kw_bar, double* kz_bar, double* scratch,
                                  hipStream_t stream, const double* s_floor) {
  if (nv < 1 || nv > GE_MAX_NV) return hipErrorInvalidValue;
  const size_t lds = geneig_lds_bytes(nv);
  switch (geneig_threads(nv)) {
    case 256:
      return launch_backward_t<256>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch, s_floor, lds,
                                    stream);
    case 512:
      return launch_backward_t<512>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch, s_floor, lds,
                                    stream);
    default:
      return launch_backward_t<GE_MAX_THREADS>(nv, ntb, k_w, k_z, g_max, tau, rho, phibar, kw_bar, kz_bar, scratch,
                                               s_floor, lds, stream);
  }
}

hipError_t launch_geneig_trace(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                               double rho, double* dos, int32_t* ranks, double* scratch, hipStream_t stream,
                               int nvh, const double* k_c, const double* trw, double* hscr,
                               const double* s_floor, int rank_stride) {
  if (nv < 1 || nv > GE_MAX_NV) return hipErrorInvalidValue;
  if (nvh < 0 || (nvh > 0 && (!k_c || !trw || !hscr))) return hipErrorInvalidValue;
  if (rank_stride <= 0) rank_stride = ntb;
  const size_t lds = geneig_lds_bytes(nv);
  switch (geneig_threads(nv)) {
    case 256:
      return launch_trace_t<256>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw, hscr,
                                 s_floor, rank_stride, lds, stream);
    case 512:
      return launch_trace_t<512>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw, hscr,
                                 s_floor, rank_stride, lds, stream);
    default:
      return launch_trace_t<GE_MAX_THREADS>(nv, ntb, k_w, k_z, g_max, tau, rho, dos, ranks, scratch, nvh, k_c, trw,
                                            hscr, s_floor, rank_stride, lds, stream);
  }
}

}  // namespace ssm
