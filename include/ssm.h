/*
 * ssm.h -- C ABI of libssm: the spectrum sweeping method (SS-DGC) for the
 * Gaussian-regularised density of states of a sparse real symmetric matrix,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: L. Lin, "Randomized estimation of spectral densities of large
 * matrices made accurate", arXiv:1504.07690.  Algorithm numbers below refer to
 * that paper.
 *
 * Conventions shared by every call
 *  - Every call returns an ssm_status; nothing is thrown across the ABI.  On
 *    error the outputs are left untouched and ssm_last_error() returns a
 *    message for the calling thread.
 *  - "device" pointers are HIP device memory owned by the caller (for example
 *    torch tensors); "host" pointers are ordinary host memory.  The library
 *    never frees or keeps caller memory beyond the documented lifetime.
 *  - The library allocates no device memory: every device buffer it needs is
 *    carved out of the workspace the caller passes to ssm_create, or is a
 *    caller buffer of a stage call.
 *  - stream is a hipStream_t (NULL = the null stream).  Stage calls only
 *    enqueue work and return; context calls that return host results
 *    synchronise the stream before returning.
 *  - Units: the matrix A, the interval [lo, hi], the sweep points t_i and the
 *    smearing sigma are all in A's own units.  The Chebyshev expansion is
 *    taken in the rescaled variable of Section 2,
 *    A~ = (2A - (lo+hi) I) / (hi - lo), whose spectrum must lie in [-1, 1].
 *  - Dense blocks are row-major: a block X of N rows and N_v columns stores
 *    X[r][j] at r*N_v + j.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef SSM_H
#define SSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ssm_status {
  SSM_OK = 0,
  SSM_ERR_ARG = 1,         /* invalid argument: null pointer, bad size, bad enum, non-finite scalar */
  SSM_ERR_WORKSPACE = 2,   /* workspace too small for any plan, or not 256-byte aligned */
  SSM_ERR_HIP = 3,         /* a HIP runtime call failed (message in ssm_last_error) */
  SSM_ERR_BOUNDS = 4,      /* ||T_M(A~)W||_F > (1 + 1e-3)||W||_F: spec(A) is not inside [lo, hi] */
  SSM_ERR_NONFINITE = 5,   /* NaN or Inf in the Gram matrices or in the DOS */
  SSM_ERR_STATE = 6,       /* call order violated (e.g. ssm_trace before ssm_dos) */
  SSM_ERR_UNSUPPORTED = 7  /* a size outside what this build implements (see each call) */
} ssm_status;

/* Arithmetic of the hot path.  In every mode the Gram matrices, the two
 * eigen-decompositions of Algorithm 4 and the trace are FP64. */
typedef enum ssm_precision {
  SSM_FP64 = 0,            /* recurrence and sweep in FP64 (CSR values double) */
  SSM_FP32 = 1,            /* recurrence and sweep in FP32 (CSR values float), FP32 MFMA sweep */
  SSM_FP32_BF16SWEEP = 2,  /* FP32 recurrence; sweep with BF16 inputs (round to nearest even)
                              and FP32 accumulation on MFMA (CSR values float) */
  SSM_FP32_BF16X3 = 3      /* FP32 recurrence; sweep with each FP32 operand split into
                              hi + lo bfloat16 terms and the three products hi.hi + hi.lo +
                              lo.hi on BF16 MFMA, FP32 accumulation (CSR values float) */
} ssm_precision;

/* Estimator run by ssm_dos. */
typedef enum ssm_method {
  SSM_SS_DGC = 0,          /* Algorithm 5: every Z(t_i) = g^M(t_i I - A~) W formed, K_W = W^T Z,
                              K_Z = Z^T Z */
  SSM_RESS_DGC = 1         /* Algorithm 7 (Theorem 4): no Z; the moments X_l = V^T T_l(A~) V of
                              V = [W W~] give K_W = sum_{l<=M/2} mu_l X_l and K_Z = sum_{l<=M}
                              nu_l X_l (nu of Proposition 1), plus the hybrid correction of
                              Algorithm 6 from the N~_v columns of W~ when nv_hybrid > 0 */
} ssm_method;

/* Sparse real symmetric matrix in CSR form, all arrays on the device and
 * borrowed for the lifetime of the context (or of the stage call). */
typedef struct ssm_csr {
  int64_t n;               /* dimension N >= 1 */
  int64_t nnz;             /* stored entries, 1 <= nnz < 2^31 */
  const int32_t* row_ptr;  /* n+1 offsets, row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz */
  const int32_t* col_idx;  /* nnz column indices in [0, n) */
  const void* values;      /* nnz values: double for SSM_FP64, float for the FP32 modes */
} ssm_csr;

/* Parameters of Algorithm 5 (with Algorithm 4's tau). */
typedef struct ssm_params {
  double lo, hi;           /* lo < hi, interval containing spec(A) (Section 2) */
  double sigma;            /* smearing sigma > 0 of g_sigma, Eq. (gaussian), A's units */
  double tau;              /* Algorithm 4 step 2 truncation, keep s_j >= tau max s; <= 0 selects 1e-7 */
  double range_slack;      /* rho: Algorithm 4 step 4 keeps xi in [0, (1+rho) g_max]; < 0 selects 1e-3 */
  int32_t nv;              /* N_v random vectors: 4 <= nv <= 256 and nv % 4 == 0 in this build */
  int32_t degree;          /* Chebyshev degree M >= 1 (T_0..T_M); M <= 4095 in this build */
  int32_t nt;              /* number of sweep points N_t >= 1 */
  int32_t precision;       /* an ssm_precision */
  uint64_t seed;           /* key of the Philox generator for W when ssm_create gets no W */
  int32_t ckpt_every;      /* s: 0, or s >= 4.  s > 0 plans for ssm_backward with a ring of fewer
                              than M+1 blocks: the first pass of ssm_dos also keeps the pairs
                              (Y_0, Y_1) and (Y_{js-1}, Y_{js}) (Y_k = T_k(A~)W, 1 <= j <= M/s),
                              from which the backward recomputes the blocks segment by segment
                              (directly into the ring when it holds s blocks, else through a
                              second level of pairs every K_c degrees) */
  int32_t dgc;             /* nonzero: ssm_dos also forms the DGC estimate of Algorithm 2 from the
                              same recurrence (same W, M and sweep points); read it with ssm_dgc
                              (SSM_SS_DGC only) */
  int32_t method;          /* an ssm_method (0 = SSM_SS_DGC).  SSM_RESS_DGC needs an even M,
                              SSM_FP64 or SSM_FP32 (else SSM_ERR_UNSUPPORTED), ckpt_every = 0
                              and dgc = 0 */
  int32_t nv_hybrid;       /* N~_v of Algorithm 7: 0, or a multiple of 4 with nv + nv_hybrid <= 256
                              (SSM_RESS_DGC only; 0 for SSM_SS_DGC).  The block W of ssm_create
                              then has nv + nv_hybrid columns: W, then W~ */
  double floor_scale;      /* eta of the rounding floor of Algorithm 4's truncation (SSM_SS_DGC):
                              step 2 also drops s_j < eta ||mu(t_i)||_2 ||W||_F^2 / sqrt(N N_v),
                              the size of the error that the sweep's rounding leaves in W^T Z(t_i)
                              (||mu(t_i)||_2 over l = 0..M).  Where Z(t_i) is below that error
                              (sweep points outside the spectrum or at its far edges) K_W and K_Z
                              are rounding and their pencil has arbitrary eigenvalues, in range
                              included; the floor keeps nothing there.  0 selects the precision's
                              default: none for SSM_FP64, 2^-22 for SSM_FP32, 2^-16 for
                              SSM_FP32_BF16X3, 2^-7 for SSM_FP32_BF16SWEEP; < 0: no floor */
  int32_t plan_batch;      /* 0: the planner chooses; > 0: sweep points per batch (pass), a
                              multiple of 8 when below nt (SSM_SS_DGC) */
  int32_t plan_chunk;      /* 0: the planner chooses; > 0: blocks in the ring (capped at M+1), a
                              multiple of 16 when below M+1 (SSM_SS_DGC).  With either set,
                              ssm_workspace_size and ssm_create return SSM_ERR_WORKSPACE when
                              that plan does not fit the budget */
  int32_t lattice[3];      /* 0, 0, 0, or (nx, ny, nz) with nx ny nz = N when row x + nx (y + ny z)
                              is point (x, y, z) of a lattice (a stencil matrix): the recurrence then
                              computes the rows tile by tile of the x-y plane, each tile through
                              every z, so that the rows a stencil gathers stay in the L2 (a
                              visiting order only: the blocks do not depend on it).  Where the
                              rows fill whole 1 KB multiples (N_v' times the element size), the
                              tiles hold multiples of 8 points and every side is at least 3, the
                              workspace also holds A's values in box order (27 N values) and, if
                              ssm_create finds every row's entries inside the 3 x 3 x 3 box of its
                              point (periodic wrap), the recurrence takes the box-stencil kernel
                              (ssm_stats.box_stencil): blocks then differ from the CSR kernel's
                              in the rounding order of rows next to the wrap only.  The values
                              in box order are refreshed from the CSR at each ssm_dos and
                              ssm_backward */
} ssm_params;

/* Per-phase device times (milliseconds, HIP events on the context's stream)
 * of the last ssm_dos, and the plan it ran. */
typedef struct ssm_stats {
  double ms_total;         /* whole ssm_dos, first launch to last kernel end */
  double ms_recurrence;    /* all Chebyshev block-SpMM launches (summed over passes) */
  double ms_sweep;         /* all sweep GEMM launches */
  double ms_gram;          /* Gram kernels incl. partial-sum reduction */
  double ms_geneig;        /* Algorithm 4 kernel */
  int64_t spmm_launches;   /* number of block-SpMM launches */
  int64_t sweep_launches;  /* number of sweep GEMM launches */
  int32_t passes;          /* recurrence passes (sweep-point batches) */
  int32_t chunk;           /* K_c: Chebyshev blocks held at once */
  int32_t batch;           /* N_t^b: sweep points per batch */
  int32_t gram_segments;   /* row segments of the Gram partial sums */
  int32_t split_k3;        /* SSM_FP32_BF16X3: degrees below this take three products (else 0) */
  int32_t box_stencil;     /* 1 if the recurrence takes the box-stencil kernel: a lattice whose
                              rows' entries all lie in the 3 x 3 x 3 box of their point (periodic
                              wrap, every side >= 3), rows of whole 1 KB multiples (N_v' times the
                              element size) and x-y tiles of a multiple of 8 points; it gathers
                              each line of a neighbourhood once for 8 points of a row of the
                              lattice and sums each point's terms in box order (the CSR order
                              away from the wrap), so blocks may differ from the CSR kernel's in
                              rounding only */
} ssm_stats;

/* Message of the last failed call on this thread ("" if none). */
const char* ssm_last_error(void);
const char* ssm_status_str(ssm_status s);

/* ------------------------------------------------------------------------
 * Context calls: the whole hot path of Algorithm 5.
 * ---------------------------------------------------------------------- */
typedef struct ssm_ctx ssm_ctx;

/* Bytes of device workspace for a plan that fits in `budget` bytes
 * (budget == 0: no limit, i.e. one recurrence pass holding every T_k(A~)W and
 * every Z(t_i)).  The plan minimises recurrence passes first, then sweep
 * read-modify-write passes.  SSM_ERR_WORKSPACE if no plan fits. */
ssm_status ssm_workspace_size(const ssm_csr* a, const ssm_params* p, size_t budget, size_t* bytes);

/* Validate, plan within ws_bytes, copy the nt sweep points t_host (A's units),
 * compute the coefficients mu_l(t_i) of Algorithm 1 on the device and, if
 * w_dev is NULL, draw W (N x N_v, entries N(0,1), Philox4x32-10 keyed by
 * p->seed, Box-Muller) into the workspace.  A non-NULL w_dev (double for
 * SSM_FP64, float otherwise) is borrowed for the context's lifetime.
 * `workspace` must be 256-byte aligned and stay valid until ssm_destroy. */
ssm_status ssm_create(const ssm_csr* a, const ssm_params* p, const double* t_host, const void* w_dev,
                      void* workspace, size_t ws_bytes, void* stream, ssm_ctx** out);

/* Algorithm 5: dos_host[i] = Tr Xi~(t_i), the SS-DGC estimate of phi_sigma(t_i)
 * (A's units).  ranks_host, if not NULL, receives 2*nt ints: r1 (eigenvalues of
 * W^T Z kept by the tau test) then r2 (generalised eigenvalues kept by the
 * range test).  Synchronises the stream. */
ssm_status ssm_dos(ssm_ctx* ctx, double* dos_host, int32_t* ranks_host);
/* With method = SSM_RESS_DGC, ssm_dos returns the RESS-DGC estimate of Algorithm 7:
 *   phi~(t_i) = Tr Xi~(t_i) + (Tr K_W~(t_i) - ||K_C(t_i) C~(t_i)||_F^2) / N~_v,
 * the second term only when nv_hybrid = N~_v > 0, with K_C = W~^T g^{M/2} W and
 * K_W~ = W~^T g^{M/2} W~ (Theorem 4).  The recurrence runs on V = [W W~] to degree
 * M/2 + 1 only: for symmetric A~, T_s^2 = (T_{2s} + T_0)/2 and T_{s+1} T_s =
 * (T_{2s+1} + T_1)/2 turn the Gram matrices of consecutive blocks into every moment
 * X_l, l <= M.  With SSM_FP64 everything is FP64; with SSM_FP32 the recurrence runs in
 * FP32 (CSR values and W float) and the Gram products and all later steps in FP64.
 * Algorithm 4's truncation also drops eigenvalues of K_W(t_i) below
 * eta sum_{l<=M/2} |mu_l(t_i)| max|X_l[:nv, :nv]|, the rounding level of K_W as a sum of
 * moments, eta = 1e-12 (SSM_FP64) or 2^-18 (SSM_FP32) (at sweep points outside the
 * spectrum K_W and K_Z are both rounding, and their pencil would otherwise report
 * arbitrary values).  ranks_host as
 * for Algorithm 5 (r1, r2 of the N_v x N_v pencil).  The bound check uses
 * ||T_{M/2+1}(A~)V||_F. */

/* Sum_i w[i] * dos[i] over the DOS of the last ssm_dos (Algorithm 8, step 4).
 * SSM_ERR_STATE before the first ssm_dos. */
ssm_status ssm_trace(ssm_ctx* ctx, const double* w_host, double* tr);

/* Algorithm 2 (DGC) on the context's W, degree M and sweep points, formed by the last
 * ssm_dos of a context made with p->dgc != 0 (SSM_ERR_STATE otherwise):
 *   zeta_l = Tr[W^T T_l(A~) W] / N_v (l = 0..M),  dgc_host[i] = sum_l mu_l(t_i) zeta_l.
 * The moments come from inner products the recurrence takes on its way (no extra pass
 * over W): the step that forms Y_{s+1} = T_{s+1}(A~)W from Y_s also sums <Y_s, Y_s> and
 * <Y_{s+1}, Y_s> (FP64 sums of the block type's products), and for symmetric A, with
 * T_s^2 = (T_{2s} + T_0)/2 and T_{s+1} T_s = (T_{2s+1} + T_1)/2,
 *   N_v zeta_{2s} = 2 <Y_s, Y_s> - N_v zeta_0,  N_v zeta_{2s+1} = 2 <Y_{s+1}, Y_s> - N_v zeta_1,
 * so only the steps s <= M/2 take them.  dgc_host: nt doubles (A's units);
 * zeta_host: NULL or M+1 doubles.  Synchronises the stream. */
ssm_status ssm_dgc(ssm_ctx* ctx, double* dgc_host, double* zeta_host);

ssm_status ssm_get_stats(const ssm_ctx* ctx, ssm_stats* out);

/* Device views of the context's buffers (valid until ssm_destroy; contents as
 * left by the last ssm_dos).  y: K_c blocks T_k(A~)W (block k at slot k mod K_c
 * of the last pass); z: the last batch's Z(t_i) blocks; k_w, k_z: nt Gram
 * matrices N_v x N_v (double); coeff: (M+1) x nt coefficients (double,
 * row-major, mu_l(t_i) at l*nt + i); w: the block W. */
typedef struct ssm_views {
  void* w; void* y; void* z; double* k_w; double* k_z; double* coeff;
  int32_t chunk; int32_t batch; int32_t first_point_of_last_batch; int32_t elem_bytes;
  double* moments;   /* SSM_RESS_DGC: X_l = V^T T_l(A~) V, l = 0..M, N_v'^2 doubles each
                        (N_v' = nv + nv_hybrid); NULL otherwise.  z is NULL and chunk
                        counts the ring's slots. */
  double* coeff_sq;  /* SSM_RESS_DGC: nu_l(t_i) of Proposition 1, same layout as coeff */
  double* s_floor;   /* SSM_SS_DGC with a rounding floor: the nt floors of the last ssm_dos
                        (see ssm_params.floor_scale); NULL otherwise */
} ssm_views;
ssm_status ssm_get_views(const ssm_ctx* ctx, ssm_views* out);

ssm_status ssm_destroy(ssm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Adjoint (not in the paper): the gradient of L = sum_i dos_bar[i] * dos[i]
 * (the DOS of the last ssm_dos) with respect to every stored value of A, each
 * value taken as an independent variable, the truncation sets of Algorithm 4
 * frozen.  For Tr f(A) ~= sum_i w_i dos[i] (Algorithm 8) pass dos_bar = w.
 *   per point:  Kbar_Z = dos_bar_i U (D P D) U^T, Kbar_W = dos_bar_i U (Gamma o
 *               (Kt D P + P D Kt)) U^T (see geneig.hip), then
 *               Zbar_i = W Kbar_W + 2 Z_i Kbar_Z;
 *   Ybar_k = sum_i mu_k(t_i) Zbar_i;
 *   Lambda_k = Ybar_k + 2 A~ Lambda_{k+1} - Lambda_{k+2} (k = M..1, Lambda_{M+1} =
 *   Lambda_{M+2} = 0);  grad[e] = alpha (Lambda_1[r_e].W[c_e] + 2 sum_{k>=2}
 *   Lambda_k[r_e].Y_{k-1}[c_e]),  alpha = 2/(hi - lo),  A symmetric.
 * Conditioning: at sweep points outside the spectrum Z_i is rounding noise, and
 * its contribution to the gradient is that noise amplified by the inverse square
 * roots of Algorithm 4 (O(1) relative in the FP32 modes).  Give such points zero
 * dos_bar (the tests and the benchmark weight points whose estimate exceeds 1e-2
 * of its maximum).
 * Arithmetic: Algorithm 4's backward and Kbar in FP64; Zbar, Ybar and Lambda in
 * the context's block type, Ybar by the context's sweep kernel; the gradient's
 * dot products and sums in FP64.
 * Needs a plan whose ring holds every T_k(A~)W or one made with ckpt_every > 0
 * (SSM_ERR_UNSUPPORTED otherwise), and a previous ssm_dos (SSM_ERR_STATE).
 * Batches: with several sweep-point batches (passes), each batch's Zbar feeds its
 * own reverse recurrence and the gradients add up (the map is linear in Ybar);
 * the batch that ssm_dos left in Z goes first, every other batch's Z is formed
 * again by the forward recurrence and sweep (bit-identical to ssm_dos's).
 * Checkpoints: T_k(A~)W of each segment of s degrees is recomputed from its
 * checkpoint pair into the context's ring (M (s-2)/s extra block products); when
 * the ring holds K_c < s blocks, a replay of the segment first keeps a pair every
 * K_c degrees in the backward workspace (about M more block products per batch).
 * The recomputed blocks are bit-identical to the forward's.  The backward
 * overwrites the context's Z blocks (and ring); a later backward forms them again.
 * grad_dev: nnz doubles (device), overwritten.  workspace: device memory of
 * at least ssm_backward_workspace_size bytes, 256-byte aligned.  Synchronises. */
ssm_status ssm_backward_workspace_size(const ssm_ctx* ctx, size_t* bytes);
ssm_status ssm_backward(ssm_ctx* ctx, const double* dos_bar_host, double* grad_dev, void* workspace,
                        size_t ws_bytes);

/* Device times (milliseconds) of the last ssm_backward: Algorithm 4 backward,
 * Zbar, transposed sweeps, recomputation of T_k(A~)W from checkpoints, reverse
 * recurrence with the SDDMM. */
typedef struct ssm_backward_stats {
  double ms_total, ms_geneig, ms_zbar, ms_ybar, ms_recompute, ms_reverse;
  int32_t segments;        /* degree segments of the reverse sweep, summed over the batches */
  int32_t recomputed;      /* blocks T_k(A~)W recomputed from checkpoints (both levels) */
  double ms_forward;       /* forward passes that regenerated Z of the other batches */
  int32_t passes;          /* sweep-point batches */
  int32_t levels;          /* 0: every block resident; 1: checkpoints; 2: two checkpoint levels */
} ssm_backward_stats;
ssm_status ssm_get_backward_stats(const ssm_ctx* ctx, ssm_backward_stats* out);

/* ------------------------------------------------------------------------
 * Algorithm 8 (host only): weights w_i with Tr f(A) ~= sum_i w_i phi~(t_i),
 * for the nt midpoints t_i = c0 + hw(-1 + (2i+1)/nt) of [lo, hi].
 * h(t) = f(t) pi(t) + c (1 - pi(t)) (Eq. hform, pi of Eq. pifunc with
 * parameters a and sigma_tilde in the rescaled variable, c = (f(x(-a)) +
 * f(x(a)))/2); f~ solves f~ * G = h periodically on the rescaled [-1, 1] with
 * G the unit-mass Gaussian of width sigma/hw, by DFT, keeping the wavenumbers
 * k with exp(-(pi k sigma/hw)^2/2) >= 1e-10; w_i = N (hi - lo)/nt f~(t_i).
 * f is called only at points where pi(t) > 1e-300, plus x(+-a).
 * Requires 0 < a < 1, sigma_tilde > 0, nt >= 2. */
typedef double (*ssm_scalar_fn)(double x, void* user);
ssm_status ssm_trace_weights(double lo, double hi, int32_t nt, int64_t n, double sigma, double a,
                             double sigma_tilde, ssm_scalar_fn f, void* user, double* w_host);

/* Algorithm 8 for f(x) = exp(-beta x) by the exact real-line deconvolution of Eq.
 * (deconvolv): G * e^{-beta s} = e^{beta^2 sigma^2/2} e^{-beta s} for the unit-mass Gaussian G
 * of width sigma, so f~(s) = e^{-beta^2 sigma^2/2} e^{-beta s} with no window and no periodic
 * extension (the exponential's periodic extension would not decay in Fourier space).
 * w_host[i] = N (hi - lo)/nt f~(t_i) on the nt midpoints of [lo, hi] (host, nt doubles),
 * and 0 where t_i < spec_lo - beta sigma^2 - 10 sigma for a lower bound spec_lo of the
 * spectrum (-INFINITY for none): the regularised DOS there is below e^{-50} of its values
 * in exact arithmetic, and for beta > 0 the weights grow like e^{-beta t}, amplifying the
 * estimate's rounding (in the FP32 modes by orders of magnitude).  Accurate when
 * (hi - lo)/nt is below sigma and [lo, hi] covers every eigenvalue minus beta sigma^2 by
 * several sigma.  SSM_ERR_ARG for non-finite or out-of-range arguments. */
ssm_status ssm_trace_weights_exp(double lo, double hi, int32_t nt, int64_t n, double sigma, double beta,
                                 double spec_lo, double* w_host);

/* ------------------------------------------------------------------------
 * Stage calls: one step of the hot path each, on caller device buffers.
 * They enqueue on `stream` and return without synchronising.
 * ---------------------------------------------------------------------- */

/* Algorithm 1 for nt points at once: c[l*nt + i] = mu_l(t_i), l = 0..M, with
 * theta_j = j pi / N_theta, 2 N_theta = least power of two >= 4(M+1), and
 * g_j = g_sigma(t_i - x(cos theta_j)), x(s) = (lo+hi)/2 + s (hi-lo)/2,
 * g_sigma of Eq. (gaussian) with its 1/N.  t_dev: nt doubles.  c32, if not
 * NULL, receives the same values rounded to float. */
ssm_status ssm_coefficients(double lo, double hi, double sigma, int64_t n, const double* t_dev,
                            int32_t nt, int32_t degree, double* c_dev, float* c32_dev, void* stream);

/* W (n x nv): element (r, j), j = 4g + m, is normal m of Philox4x32-10 with
 * counter (g, 0, r mod 2^32, r div 2^32) and key (seed mod 2^32, seed div
 * 2^32); Box-Muller with u = (x0+1) 2^-32, v = x1 2^-32 (normals 0, 1 =
 * sqrt(-2 ln u) cos/sin(2 pi v)) and likewise (x2, x3) for normals 2, 3.
 * Computed in double; dtype 0 stores double, 1 stores float. */
ssm_status ssm_gaussian_block(uint64_t seed, int64_t n, int32_t nv, int32_t dtype, void* w_dev,
                              void* stream);

/* The three-term recurrence of Algorithm 5 (steps 3, 9, 10):
 * y holds M+1 consecutive blocks (n x nv each); block 0 <- w,
 * block 1 <- A~ w, block k+1 <- 2 A~ block k - block k-1, with
 * A~ = (2A - (lo+hi) I)/(hi-lo).  FP64 when precision == SSM_FP64, else FP32. */
ssm_status ssm_chebyshev(const ssm_csr* a, double lo, double hi, int32_t precision, int32_t nv,
                         int32_t degree, const void* w, void* y, void* stream);

/* The sweep (Algorithm 5, steps 6-8) over a chunk of kc blocks and ntb points:
 * z[i*e + q] (+)= sum_{k<kc} c[k*ldc + i] * y[k*e + q],  i < ntb, q < e,
 * with e = N * N_v elements per block.  accumulate = 0 overwrites z.
 * SSM_FP64: c, y, z double (FP64 MFMA).  SSM_FP32: c, y, z float (FP32 MFMA).
 * SSM_FP32_BF16SWEEP: c, y, z float; c and y rounded to bfloat16 (nearest
 * even) before the products, FP32 accumulation (BF16 MFMA).  SSM_FP32_BF16X3
 * takes split tables: use ssm_split_coefficients and ssm_sweep_split. */
ssm_status ssm_sweep(int32_t precision, int64_t e, int32_t kc, int32_t ntb, const void* c, int64_t ldc,
                     const void* y, void* z, int32_t accumulate, void* stream);

/* Split coefficient table for SSM_FP32_BF16X3: for i < nt, l < m1,
 * chi[i*ldk + l] = bf16(c[l*ldc + i]) and clo[i*ldk + l] = bf16(c[l*ldc + i] - chi),
 * each rounded once from the double value to the nearest bfloat16 (ties to even);
 * entries with l >= m1 are 0.  c: m1 x ldc doubles;
 * chi, clo: nt x ldk bfloat16 (2 bytes), ldk >= m1, ldk % 8 == 0, 16-byte aligned. */
ssm_status ssm_split_coefficients(const double* c, int64_t ldc, int32_t nt, int32_t m1, void* chi, void* clo,
                                  int64_t ldk, void* stream);

/* The sweep of ssm_sweep in the SSM_FP32_BF16X3 arithmetic:
 * z[i*e + q] (+)= sum_{k<kc} c[k][i] y[k*e + q] with c given by its split tables
 * (row i at chi + i*ldk, k = 0..kc-1 from the pointer; ldk % 8 == 0; chi, clo, y
 * and z 16-byte aligned; of row ntb-1 the first kc entries rounded up to a multiple of 8
 * are read, and ntb*ldk must stay below 2^30 entries); y and z float, e % 4 == 0;
 * SSM_ERR_ARG otherwise.  ldk % 64 == 0 (128-byte rows) is the fastest stride: the
 * kernel reads 64-byte pieces of each row, which then never straddle two cache lines.
 * k3: degrees k < k3 (rounded up to a multiple of 32) take the three products
 * Chi^T Yhi + Chi^T Ylo + Clo^T Yhi, the others Chi^T Yhi alone; k3 >= kc: three
 * everywhere.  ssm_dos sets k3 one past the last degree whose coefficients reach
 * 2^-8 of the table's largest: beyond it the single product's relative rounding
 * (<= 2^-8) stays under 2^-16 of the largest term, the level the three products
 * leave on the leading degrees (the Gaussian's coefficients decay like
 * exp(-(k sigma^)^2/2), so the tail is most of the table). */
ssm_status ssm_sweep_split(int64_t e, int32_t kc, int32_t ntb, const void* chi, const void* clo, int64_t ldk,
                           const void* y, void* z, int32_t accumulate, int32_t k3, void* stream);

/* Gram matrices of ntb sweep points (Eq. tracelr, Algorithm 5 step 13):
 * k_w[i] = the symmetric completion of W^T Z_i from its upper 16 x 16 blocks: entry
 * (r, c) of block (a, b), a < b, is (W^T Z_i)[r][c] and is mirrored to (c, r); diagonal
 * blocks are ((W^T Z_i) + (W^T Z_i)^T)/2.  W^T Z_i is symmetric in exact arithmetic on
 * the method's path (Z_i = g(t_i I - A) W, A symmetric), where this equals
 * (W^T Z_i + Z_i^T W)/2 up to rounding with one block product less.
 * k_z[i] = Z_i^T Z_i  (nv x nv doubles each), Z_i = z + i*n*nv.
 * Products and sums in FP64 (FP32 inputs widened exactly).
 * w, z: double for SSM_FP64, float otherwise.  The rows are split in nseg
 * segments, each walked by four waves whose partial sums go to `scratch`
 * (4*nseg*ntb*2*nv*nv doubles)
 * and are then added in a fixed order (deterministic). */
ssm_status ssm_gram(int32_t precision, int64_t n, int32_t nv, int32_t ntb, const void* w, const void* z,
                    double* k_w, double* k_z, int32_t nseg, double* scratch, void* stream);

/* ssm_gram for callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same computation and result,
 * with no scratch argument.  The partial sums go to a device array of
 * SSM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends; its address is looked up on the first call on each device (with the
 * current device being the one stream runs on).  The call allocates nothing.
 * SSM_ERR_UNSUPPORTED when the partial sums, 4 nseg ntb 2 nv^2 doubles, exceed the array.
 * Every call on one GPU shares that GPU's array and leaves its own partial sums in it
 * (each call writes every partial sum it reads, so nothing needs clearing): calls on one
 * stream are ordered, but calls that overlap on one GPU (other streams, other threads)
 * race. */
#define SSM_NOALLOC_SCRATCH_BYTES (32 << 20)
ssm_status ssm_gram_noalloc(int32_t precision, int64_t n, int32_t nv, int32_t ntb, const void* w, const void* z,
                            double* k_w, double* k_z, int32_t nseg, void* stream);

/* Algorithm 4 and the trace, for ntb points: for point i, eig(k_w[i]) = U S U^T
 * (k_w[i] taken as its symmetric part), keep s_j >= tau max_j s_j (nothing if
 * max s <= 0), B = S~^-1/2 U~^T k_z[i] U~ S~^-1/2, eig(B) = xi, dos[i] = sum of xi
 * in [0, (1 + rho) g_max]; ranks[i] = r1, ranks[ntb + i] = r2 (ranks may be NULL).
 * All in FP64: cyclic Jacobi for nv <= 48; above, a Householder reduction to
 * tridiagonal form, implicit QL for eig(k_w[i]) and bisection for eig(B) (a point
 * whose QL iterations run past their limit is redone by Jacobi).  k_w, k_z: ntb
 * row-major nv x nv FP64 matrices on the device; dos_dev: ntb doubles, ranks_dev:
 * 2 ntb int32 (may be NULL).  scratch: ssm_geneig_trace_scratch_doubles(nv, ntb)
 * doubles of device memory, owned by the caller, contents ignored on entry.
 * SSM_ERR_ARG on NULL pointers, nv or ntb < 1 or bad g_max/tau/rho;
 * SSM_ERR_UNSUPPORTED for nv > 256. */
ssm_status ssm_geneig_trace(int32_t nv, int32_t ntb, const double* k_w, const double* k_z, double g_max,
                            double tau, double rho, double* dos_dev, int32_t* ranks_dev, double* scratch,
                            void* stream);
/* Scratch of ssm_geneig_trace in doubles: ntb nv^2 for nv <= 48, min(ntb, 2048)
 * (6 nv^2 + 8 nv + 8) above (the tridiagonal path runs 2048 points at a time).  -1 for
 * nv outside [1, 256] or ntb < 1. */
int64_t ssm_geneig_trace_scratch_doubles(int32_t nv, int32_t ntb);

#ifdef __cplusplus
}
#endif
#endif /* SSM_H */
