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
// The matrix and its eigenvectors live in LDS (N_v <= 96: 2 * 96 * 97 doubles);
// the N_v x r1 product Z^T Z U~ S~^-1/2 goes through a per-point global scratch.
#include "ssm_kernels.h"

namespace ssm {
namespace {

constexpr int GE_THREADS = 256;
constexpr int GE_MAX_NV = 96;
constexpr int GE_MAX_SWEEPS = 40;

struct GeShared {
  double* A;      // n x ld
  double* V;      // n x ld
  double* s;      // eigenvalues
  double* scale;  // s^-1/2 of kept ones
  double* cs;     // pair cosines
  double* sn;     // pair sines
  double* red;    // reduction scratch (GE_THREADS)
  int* pp;        // pair rows
  int* qq;        // pair cols
  int* kidx;      // kept indices
  int* misc;      // [0] = r1
};

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int st = GE_THREADS / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Diagonalise the symmetric n x n matrix in sh.A (row stride ld); accumulate the
// rotations into V (if V != nullptr, V must hold the identity on entry).
__device__ void jacobi(const GeShared& sh, double* V, int n, int ld) {
  double* A = sh.A;
  const int tid = threadIdx.x;
  const int ne = n + (n & 1);
  const int npairs = ne / 2;
  for (int sweep = 0; sweep < GE_MAX_SWEEPS; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int idx = tid; idx < n * n; idx += GE_THREADS) {
      const int r = idx / n, c = idx - r * n;
      const double v = A[r * ld + c];
      all += v * v;
      if (r != c) off += v * v;
    }
    off = block_sum(off, sh.red);
    all = block_sum(all, sh.red);
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
        } else {
          p = -1;
          q = -1;
        }
        sh.pp[tid] = p;
        sh.qq[tid] = q;
        sh.cs[tid] = c;
        sh.sn[tid] = s;
      }
      __syncthreads();
      // rows: A <- J^T A  (row p <- c row_p - s row_q, row q <- s row_p + c row_q)
      for (int idx = tid; idx < npairs * n; idx += GE_THREADS) {
        const int j = idx / n, col = idx - j * n;
        const int p = sh.pp[j], q = sh.qq[j];
        if (p < 0) continue;
        const double c = sh.cs[j], s = sh.sn[j];
        const double ap = A[p * ld + col], aq = A[q * ld + col];
        A[p * ld + col] = c * ap - s * aq;
        A[q * ld + col] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J; the pivot pair (p,q),(q,p) becomes exactly 0
      for (int idx = tid; idx < npairs * n; idx += GE_THREADS) {
        const int j = idx / n, row = idx - j * n;
        const int p = sh.pp[j], q = sh.qq[j];
        if (p < 0) continue;
        const double c = sh.cs[j], s = sh.sn[j];
        const double ap = A[row * ld + p], aq = A[row * ld + q];
        A[row * ld + p] = (row == q) ? 0.0 : c * ap - s * aq;
        A[row * ld + q] = (row == p) ? 0.0 : s * ap + c * aq;
        if (V) {
          const double vp = V[row * ld + p], vq = V[row * ld + q];
          V[row * ld + p] = c * vp - s * vq;
          V[row * ld + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(GE_THREADS) geneig_trace_kernel(int nv, const double* __restrict__ k_w,
                                                                  const double* __restrict__ k_z, double g_max,
                                                                  double tau, double rho, double* __restrict__ dos,
                                                                  int32_t* __restrict__ ranks, int ntb,
                                                                  double* __restrict__ scratch) {
  extern __shared__ double lds[];
  const int n = nv;
  const int ld = n + 1;
  GeShared sh;
  sh.A = lds;
  sh.V = sh.A + n * ld;
  sh.s = sh.V + n * ld;
  sh.scale = sh.s + GE_MAX_NV;
  sh.cs = sh.scale + GE_MAX_NV;
  sh.sn = sh.cs + GE_MAX_NV / 2;
  sh.red = sh.sn + GE_MAX_NV / 2;
  sh.pp = (int*)(sh.red + GE_THREADS);
  sh.qq = sh.pp + GE_MAX_NV / 2;
  sh.kidx = sh.qq + GE_MAX_NV / 2;
  sh.misc = sh.kidx + GE_MAX_NV;

  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  const double* kw = k_w + i * nn;
  const double* kz = k_z + i * nn;
  double* tmat = scratch + i * nn;

  for (int idx = tid; idx < n * n; idx += GE_THREADS) {
    const int r = idx / n, c = idx - r * n;
    sh.A[r * ld + c] = kw[idx];
    sh.V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // 1. W^T Z = U S U^T
  jacobi(sh, sh.V, n, ld);
  for (int j = tid; j < n; j += GE_THREADS) sh.s[j] = sh.A[j * ld + j];
  __syncthreads();

  // 2. truncation
  if (tid == 0) {
    double smax = -INFINITY;
    for (int j = 0; j < n; ++j) smax = fmax(smax, sh.s[j]);
    int r1 = 0;
    if (smax > 0.0) {
      const double thr = tau * smax;
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
      dos[i] = 0.0;
      if (ranks) {
        ranks[i] = 0;
        ranks[ntb + i] = 0;
      }
    }
    return;
  }

  // 3a. T = (Z^T Z) U~ S~^-1/2   (n x r1, global scratch, row stride r1)
  for (int idx = tid; idx < n * r1; idx += GE_THREADS) {
    const int row = idx / r1, a = idx - row * r1;
    const int ka = sh.kidx[a];
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += kz[(int64_t)row * n + c] * sh.V[c * ld + ka];
    tmat[idx] = acc * sh.scale[a];
  }
  __threadfence_block();
  __syncthreads();
  // 3b. B = S~^-1/2 U~^T T  -> A (r1 x r1)
  for (int idx = tid; idx < r1 * r1; idx += GE_THREADS) {
    const int a = idx / r1, b = idx - a * r1;
    const int ka = sh.kidx[a];
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += sh.V[c * ld + ka] * tmat[(int64_t)c * r1 + b];
    sh.A[a * ld + b] = acc * sh.scale[a];
  }
  __syncthreads();
  for (int idx = tid; idx < r1 * r1; idx += GE_THREADS) {
    const int a = idx / r1, b = idx - a * r1;
    if (a < b) {
      const double m = 0.5 * (sh.A[a * ld + b] + sh.A[b * ld + a]);
      sh.A[a * ld + b] = m;
      sh.A[b * ld + a] = m;
    }
  }
  __syncthreads();
  jacobi(sh, nullptr, r1, ld);

  // 4. range filter and trace (fixed order)
  if (tid == 0) {
    const double hi = (1.0 + rho) * g_max;
    double tr = 0.0;
    int r2 = 0;
    for (int j = 0; j < r1; ++j) {
      const double xi = sh.A[j * ld + j];
      if (xi >= 0.0 && xi <= hi) {
        tr += xi;
        ++r2;
      }
    }
    dos[i] = tr;
    if (ranks) {
      ranks[i] = r1;
      ranks[ntb + i] = r2;
    }
  }
}

}  // namespace

size_t geneig_lds_bytes(int nv) {
  const size_t n = (size_t)nv, ld = n + 1;
  return (2 * n * ld + 2 * GE_MAX_NV + GE_MAX_NV + GE_THREADS) * sizeof(double) +
         (GE_MAX_NV + GE_MAX_NV + 4) * sizeof(int);
}

hipError_t launch_geneig_trace(int nv, int ntb, const double* k_w, const double* k_z, double g_max, double tau,
                               double rho, double* dos, int32_t* ranks, double* scratch, hipStream_t stream) {
  if (nv < 1 || nv > GE_MAX_NV) return hipErrorInvalidValue;
  const size_t lds = geneig_lds_bytes(nv);
  hipError_t err = hipFuncSetAttribute((const void*)geneig_trace_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(geneig_trace_kernel, dim3(ntb), dim3(GE_THREADS), lds, stream, nv, k_w, k_z, g_max, tau, rho,
                     dos, ranks, ntb, scratch);
  return hipGetLastError();
}

}  // namespace ssm
