// libssm host side: argument validation, workspace planning, the driver of
// Algorithm 5 on the device, the stage calls, and the weights of Algorithm 8.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ssm.h"
#include "ssm_kernels.h"

namespace {

thread_local std::string g_last_error;

ssm_status fail(ssm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

ssm_status hip_fail(hipError_t e, const char* what) {
  return fail(SSM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define SSM_HIP(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Scratch of ssm_gram_noalloc: the Gram kernel's partial sums, in a device array that
// every GPU the library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device address): the
// address comes from hipGetSymbolAddress, once per device with that device current.
static __device__ __align__(256) double scratch[SSM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

ssm_status noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SSM_ERR_UNSUPPORTED, "device %d beyond the %d handled", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
    if (!p) return fail(SSM_ERR_HIP, "hipGetSymbolAddress gave no address for the scratch array");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return SSM_OK;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kMaxNv = 256;
constexpr int kMaxDegree = 4095;
constexpr int kMinChunk = 16;

int n_theta_for(int degree) {
  int two = 1;
  while (two < 4 * (degree + 1)) two *= 2;
  return two / 2;
}

size_t elem_bytes(int precision) { return precision == SSM_FP64 ? 8 : 4; }

ssm_status check_csr(const ssm_csr* a) {
  if (!a) return fail(SSM_ERR_ARG, "csr is NULL");
  if (a->n < 1) return fail(SSM_ERR_ARG, "csr.n must be >= 1 (got %lld)", (long long)a->n);
  if (a->nnz < 1 || a->nnz >= 0x7FFFFFFFLL) return fail(SSM_ERR_ARG, "csr.nnz must be in [1, 2^31)");
  if (a->n > (int64_t)1 << 31) return fail(SSM_ERR_UNSUPPORTED, "csr.n above 2^31");
  if (!a->row_ptr || !a->col_idx || !a->values) return fail(SSM_ERR_ARG, "csr arrays must be non-NULL");
  return SSM_OK;
}

ssm_status check_params(const ssm_params* p) {
  if (!p) return fail(SSM_ERR_ARG, "params is NULL");
  if (!std::isfinite(p->lo) || !std::isfinite(p->hi) || !(p->lo < p->hi))
    return fail(SSM_ERR_ARG, "need finite lo < hi (got %g, %g)", p->lo, p->hi);
  if (!std::isfinite(p->sigma) || !(p->sigma > 0)) return fail(SSM_ERR_ARG, "sigma must be finite and > 0");
  if (!std::isfinite(p->tau) || !std::isfinite(p->range_slack)) return fail(SSM_ERR_ARG, "tau, rho must be finite");
  if (!std::isfinite(p->floor_scale)) return fail(SSM_ERR_ARG, "floor_scale must be finite");
  if (p->tau >= 1.0) return fail(SSM_ERR_ARG, "tau must be < 1");
  if (p->nv < 4 || p->nv % 4 != 0) return fail(SSM_ERR_ARG, "nv must be a positive multiple of 4 (got %d)", p->nv);
  if (p->nv > kMaxNv) return fail(SSM_ERR_UNSUPPORTED, "nv > %d is not implemented in this build", kMaxNv);
  if (p->degree < 1) return fail(SSM_ERR_ARG, "degree must be >= 1");
  if (p->degree > kMaxDegree) return fail(SSM_ERR_UNSUPPORTED, "degree > %d is not implemented", kMaxDegree);
  if (p->nt < 1) return fail(SSM_ERR_ARG, "nt must be >= 1");
  if (p->precision < SSM_FP64 || p->precision > SSM_FP32_BF16X3)
    return fail(SSM_ERR_ARG, "unknown precision %d", p->precision);
  if (p->ckpt_every != 0 && p->ckpt_every < 4) return fail(SSM_ERR_ARG, "ckpt_every must be 0 or >= 4");
  if (p->plan_batch < 0 || p->plan_chunk < 0) return fail(SSM_ERR_ARG, "plan_batch and plan_chunk must be >= 0");
  const int32_t* lt = p->lattice;
  if ((lt[0] || lt[1] || lt[2]) && !(lt[0] > 0 && lt[1] > 0 && lt[2] > 0))
    return fail(SSM_ERR_ARG, "lattice must be all 0 or all positive");
  if (p->plan_batch > 0 && p->plan_batch < p->nt && p->plan_batch % 8)
    return fail(SSM_ERR_ARG, "plan_batch below nt must be a multiple of 8 (got %d)", p->plan_batch);
  if (p->plan_chunk > 0 && p->plan_chunk <= p->degree && p->plan_chunk % kMinChunk)
    return fail(SSM_ERR_ARG, "plan_chunk below M+1 must be a multiple of %d (got %d)", kMinChunk, p->plan_chunk);
  if (p->method != SSM_SS_DGC && p->method != SSM_RESS_DGC) return fail(SSM_ERR_ARG, "unknown method %d", p->method);
  if (p->method == SSM_SS_DGC) {
    if (p->nv_hybrid != 0) return fail(SSM_ERR_ARG, "nv_hybrid applies to SSM_RESS_DGC only");
  } else {
    if (p->degree % 2) return fail(SSM_ERR_ARG, "RESS-DGC needs an even degree (Proposition 1), got %d", p->degree);
    if (p->nv_hybrid < 0 || p->nv_hybrid % 4)
      return fail(SSM_ERR_ARG, "nv_hybrid must be 0 or a positive multiple of 4 (got %d)", p->nv_hybrid);
    if (p->nv + p->nv_hybrid > kMaxNv)
      return fail(SSM_ERR_UNSUPPORTED, "nv + nv_hybrid > %d is not implemented in this build", kMaxNv);
    if (p->precision != SSM_FP64 && p->precision != SSM_FP32)
      return fail(SSM_ERR_UNSUPPORTED, "RESS-DGC runs in FP64 or FP32 in this build");
    if (p->ckpt_every) return fail(SSM_ERR_UNSUPPORTED, "RESS-DGC has no adjoint in this build (ckpt_every must be 0)");
    if (p->dgc) return fail(SSM_ERR_UNSUPPORTED, "the DGC by-product is built for SSM_SS_DGC only");
    if (p->plan_batch || p->plan_chunk) return fail(SSM_ERR_ARG, "plan_batch and plan_chunk apply to SSM_SS_DGC");
  }
  return SSM_OK;
}

ssm_status check_lattice(const ssm_csr* a, const ssm_params* p) {
  const int32_t* lt = p->lattice;
  if (lt[0] && (int64_t)lt[0] * lt[1] * lt[2] != a->n)
    return fail(SSM_ERR_ARG, "lattice %d x %d x %d does not have n = %lld points", lt[0], lt[1], lt[2],
                (long long)a->n);
  return SSM_OK;
}

// The recurrence's visiting order for a lattice: tiles of the largest power of two up to
// 16 that divides each of nx and ny (plain row order without a lattice).
ssm::RowOrder row_order(const ssm_params* p) {
  ssm::RowOrder o;
  if (!p->lattice[0]) return o;
  auto tile = [](int n) {
    int t = 16;
    while (n % t) t /= 2;
    return t;
  };
  o.nx = p->lattice[0];
  o.ny = p->lattice[1];
  o.nz = p->lattice[2];
  o.tx = tile(o.nx);
  o.ty = tile(o.ny);
  return o;
}

// Bytes of A's values in box order that a context keeps when its lattice rows fill whole
// waves (N_v' values of a row take a multiple of 1 KB) and its tiles hold whole groups of
// kBoxRows points: the recurrence may then take the box kernel (if A's pattern passes the
// box check at ssm_create).  0 otherwise.
size_t box_bytes(const ssm_csr* a, const ssm_params* p) {
  if (!p->lattice[0]) return 0;
  const ssm::RowOrder o = row_order(p);
  const size_t es = elem_bytes(p->precision);
  const int nvp = p->nv + (p->method == SSM_RESS_DGC ? p->nv_hybrid : 0);
  if (o.nx < 3 || o.ny < 3 || o.nz < 3 || o.tx % ssm::kBoxRows || (nvp * es) % 1024) return 0;
  return (size_t)a->n * 27 * es;
}

double eff_tau(const ssm_params* p) { return p->tau > 0 ? p->tau : 1e-7; }
double eff_rho(const ssm_params* p) { return p->range_slack >= 0 ? p->range_slack : 1e-3; }

// eta of the rounding floor of Algorithm 4's truncation (SS-DGC): about two to four times the
// relative rounding that one term mu_l(t_i) T_l(A~)W of the sweep carries in the precision's
// arithmetic (FP32 products and blocks 2^-24; split BF16 about 2^-17 on the three-product
// degrees and below 2^-16 of the largest term on the others; BF16 operands 2^-8).  FP64 takes
// none: its floor would sit far below the tau test.
double eff_floor_scale(const ssm_params* p) {
  if (p->method != SSM_SS_DGC || p->floor_scale < 0) return 0.0;
  if (p->floor_scale > 0) return p->floor_scale;
  switch (p->precision) {
    case SSM_FP32: return std::ldexp(1.0, -22);
    case SSM_FP32_BF16X3: return std::ldexp(1.0, -16);
    case SSM_FP32_BF16SWEEP: return std::ldexp(1.0, -7);
    default: return 0.0;
  }
}

struct Plan {
  int passes = 1, chunk = 1, batch = 1, nseg = 1;
  int ckpt = 0;  // checkpoint interval s when the ring holds fewer than M+1 blocks, else 0
  int64_t ldc = 4, ldk = 8;
  size_t off_t = 0, off_c64 = 0, off_c32 = 0, off_chi = 0, off_clo = 0, off_w = 0, off_y = 0, off_z = 0, off_kw = 0, off_kz = 0,
         off_gpart = 0, off_escr = 0, off_dos = 0, off_ranks = 0, off_norm = 0, off_ckpt = 0, off_dpart = 0,
         off_dsums = 0, off_dgc = 0, total = 0;
  int dgc_group = 0;  // recurrence steps whose inner-product partials are held at once (0: no DGC)
  // RESS-DGC: chunk = new blocks per round, ring of chunk + 1 slots
  bool ress = false;
  size_t off_nu = 0, off_kc = 0, off_trw = 0, off_hscr = 0, off_pw = 0, off_pz = 0, off_x = 0, off_kmu = 0,
         off_knu = 0, off_xmax = 0, off_floor = 0, off_mun = 0, off_kmax = 0;
  size_t off_box = 0, box_bytes = 0;  // A's values in box order (lattice box stencils)
};

// Algorithm 2 by-product: recurrence steps s = 0..M/2 take inner products; their
// workgroup partials are reduced a group of steps at a time (at most 64 steps or 256 MiB).
int dgc_steps(int degree) { return degree / 2 + 1; }
int dgc_group(const ssm_csr* a, const ssm_params* p) {
  if (!p->dgc) return 0;
  const int64_t per_step = 2 * ssm::cheb_step_blocks(a->n, p->nv, p->precision != SSM_FP64) * 8;
  const int64_t fit = std::max<int64_t>(1, (int64_t(256) << 20) / per_step);
  return (int)std::min<int64_t>({(int64_t)64, fit, (int64_t)dgc_steps(p->degree)});
}

// Split BF16: one past the last degree whose coefficients reach 2^-8 of the table's
// largest coefficient, from the largest |mu_l(t_i)| of each degree l; degrees below it take
// the three products, the rest one.
int three_product_degrees(const std::vector<double>& kmax) {
  double cmax = 0.0;
  for (double v : kmax) cmax = std::max(cmax, v);
  int k3 = 0;
  for (size_t k = 0; k < kmax.size(); ++k)
    if (kmax[k] >= std::ldexp(cmax, -8)) k3 = (int)k + 1;
  return k3;
}

// Checkpoint pairs: (Y_0, Y_1), then (Y_{js-1}, Y_{js}) for 1 <= j <= M/s.
int ckpt_pairs(int degree, int s) { return degree / s + 1; }
int ckpt_first(int j, int s) { return j == 0 ? 0 : j * s - 1; }

// Row segments of the Gram: enough (point, segment) workgroups to cover the 256 CUs a few
// times, each wave keeping at least 64 rows.
int gram_segments(int64_t n, int batch) {
  int s = (int)std::min<int64_t>(64, std::max<int64_t>(1, (1024 + batch - 1) / batch));
  while (s > 1 && n / s < 256) --s;
  return s;
}

void layout(Plan& pl, const ssm_csr* a, const ssm_params* p, bool own_w) {
  const size_t es = elem_bytes(p->precision);
  const size_t e = (size_t)a->n * p->nv;
  const size_t nn = (size_t)p->nv * p->nv;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align_up(bytes);
    return r;
  };
  pl.off_t = take(p->nt * 8);
  pl.off_c64 = take((size_t)(p->degree + 1) * pl.ldc * 8);
  pl.off_c32 = take(p->precision == SSM_FP64 ? 0 : (size_t)(p->degree + 1) * pl.ldc * 4);
  const bool split = p->precision == SSM_FP32_BF16X3;
  pl.off_chi = take(split ? (size_t)p->nt * pl.ldk * 2 : 0);
  pl.off_clo = take(split ? (size_t)p->nt * pl.ldk * 2 : 0);
  pl.off_w = take(own_w ? e * es : 0);
  pl.off_kw = take((size_t)p->nt * nn * 8);
  pl.off_kz = take((size_t)p->nt * nn * 8);
  pl.off_escr = take((size_t)ssm::geneig_trace_scratch_doubles(p->nv, p->nt) * 8);
  pl.off_dos = take(p->nt * 8);
  pl.off_ranks = take(2 * (size_t)p->nt * 4);
  pl.off_norm = take((size_t)(ssm::reduce_partials() + 8) * 8);
  pl.off_mun = take((size_t)p->nt * 8);
  pl.off_floor = take((size_t)p->nt * 8);
  pl.off_kmax = take(split ? (size_t)(p->degree + 1) * 8 : 0);
  pl.off_gpart = take((size_t)ssm::gram_scratch_slots(pl.nseg) * pl.batch * 2 * nn * 8);
  pl.off_z = take((size_t)pl.batch * e * es);
  pl.off_y = take((size_t)pl.chunk * e * es);
  pl.ckpt = (p->ckpt_every > 0 && pl.chunk < p->degree + 1) ? p->ckpt_every : 0;
  pl.off_ckpt = take(pl.ckpt ? (size_t)2 * ckpt_pairs(p->degree, pl.ckpt) * e * es : 0);
  pl.dgc_group = dgc_group(a, p);
  pl.off_dpart = take(pl.dgc_group ? (size_t)pl.dgc_group * 2 *
                                         ssm::cheb_step_blocks(a->n, p->nv, p->precision != SSM_FP64) * 8
                                   : 0);
  pl.off_dsums = take(pl.dgc_group ? (size_t)2 * dgc_steps(p->degree) * 8 : 0);
  pl.off_dgc = take(pl.dgc_group ? (size_t)(p->nt + p->degree + 1) * 8 : 0);
  pl.box_bytes = box_bytes(a, p);
  pl.off_box = take(pl.box_bytes);
  pl.total = o;
}

// RESS-DGC: blocks Y_0..Y_S of V = [W W~] (S = M/2 + 1) in a ring of chunk + 1 slots,
// the pair Gram matrices of s = 0..S-1, the moments X_0..X_M, K_mu and K_nu per point.
void layout_ress(Plan& pl, const ssm_csr* a, const ssm_params* p, bool own_w) {
  const int nvp = p->nv + p->nv_hybrid;
  const size_t e = (size_t)a->n * nvp;
  const size_t es = elem_bytes(p->precision);
  const size_t nn = (size_t)p->nv * p->nv;
  const size_t nnp = (size_t)nvp * nvp;
  const int m1 = p->degree + 1;
  const int S = p->degree / 2 + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align_up(bytes);
    return r;
  };
  pl.off_t = take(p->nt * 8);
  pl.off_c64 = take((size_t)m1 * pl.ldc * 8);
  pl.off_nu = take((size_t)m1 * pl.ldc * 8);
  pl.off_w = take(own_w ? e * es : 0);
  pl.off_kw = take((size_t)p->nt * nn * 8);
  pl.off_kz = take((size_t)p->nt * nn * 8);
  pl.off_kc = take((size_t)p->nt * p->nv_hybrid * p->nv * 8);
  pl.off_trw = take((size_t)p->nt * 8);
  pl.off_hscr = take((size_t)p->nt * p->nv_hybrid * p->nv * 8);
  pl.off_escr = take((size_t)ssm::geneig_trace_scratch_doubles(p->nv, p->nt) * 8);
  pl.off_dos = take(p->nt * 8);
  pl.off_ranks = take(2 * (size_t)p->nt * 4);
  pl.off_norm = take((size_t)(ssm::reduce_partials() + 8) * 8);
  pl.off_pw = take((size_t)S * nnp * 8);
  pl.off_pz = take((size_t)S * nnp * 8);
  pl.off_x = take((size_t)m1 * nnp * 8);
  pl.off_kmu = take((size_t)p->nt * nnp * 8);
  pl.off_knu = take((size_t)p->nt * nnp * 8);
  pl.off_xmax = take((size_t)S * 8);
  pl.off_floor = take((size_t)p->nt * 8);
  pl.off_gpart = take((size_t)ssm::gram_scratch_slots(pl.nseg) * std::max(pl.chunk, 1) * 2 * nnp * 8);
  pl.off_y = take((size_t)(pl.chunk + 1) * e * es);
  pl.box_bytes = box_bytes(a, p);
  pl.off_box = take(pl.box_bytes);
  pl.total = o;
}

ssm_status make_plan_ress(const ssm_csr* a, const ssm_params* p, bool own_w, size_t budget, Plan& out) {
  const int S = p->degree / 2 + 1;
  Plan pl;
  pl.ress = true;
  pl.passes = 1;
  pl.batch = p->nt;
  pl.ldc = (p->nt + 3) / 4 * 4;
  for (int chunk = S; chunk >= 2; --chunk) {  // the ring keeps Y_{k-1}, Y_{k-2} and a round's first pair
    pl.chunk = chunk;
    pl.nseg = gram_segments(a->n, chunk);
    layout_ress(pl, a, p, own_w);
    if (!budget || pl.total <= budget) {
      out = pl;
      return SSM_OK;
    }
  }
  return fail(SSM_ERR_WORKSPACE, "no RESS-DGC plan fits in %zu bytes of workspace", budget);
}

// Minimise modelled bytes: recurrence replays (one per pass) against read-modify-write
// of the Z batch for every extra chunk.
ssm_status make_plan(const ssm_csr* a, const ssm_params* p, bool own_w, size_t budget, Plan& out) {
  if (p->method == SSM_RESS_DGC) return make_plan_ress(a, p, own_w, budget, out);
  const size_t es = elem_bytes(p->precision);
  const double e = (double)a->n * p->nv;
  const double spmm_bytes = 3.0 * e * es + (double)a->nnz * (4.0 + es);
  Plan best;
  double best_cost = -1.0;
  const int m1 = p->degree + 1;
  const int forced_passes = p->plan_batch > 0 ? (p->nt + p->plan_batch - 1) / p->plan_batch : 0;
  for (int passes = forced_passes ? forced_passes : 1; passes <= p->nt; ++passes) {
    int batch = (p->nt + passes - 1) / passes;
    // batch starts stay 16-byte aligned in the coefficient tables (the adjoint's transposed
    // BF16 tables hold the points of a degree contiguously)
    if (passes > 1) batch = (batch + 7) / 8 * 8;
    if (forced_passes) batch = std::min(p->plan_batch, p->nt);
    if ((p->nt + batch - 1) / batch != passes) continue;  // same batch as a smaller pass count
    Plan pl;
    pl.ldc = (p->nt + 3) / 4 * 4;
    // rows of the split tables start on 128-byte lines, so the sweep's 64-byte pieces of a
    // row never straddle two lines (a quarter of them did at a 2016-byte stride: 3% slower)
    pl.ldk = (m1 + 63) / 64 * 64;
    pl.passes = passes;
    pl.batch = batch;
    pl.nseg = gram_segments(a->n, batch);
    pl.chunk = 0;
    layout(pl, a, p, own_w);
    const size_t fixed = pl.total;
    int chunk = p->plan_chunk > 0 ? std::min(p->plan_chunk, m1) : m1;
    if (budget && !p->plan_chunk) {
      const double room = (double)budget - (double)fixed;
      chunk = room > 0 ? (int)std::min<double>(m1, std::floor(room / ((double)e * es))) : 0;
      for (; chunk >= 1; --chunk) {  // the ring's size is rounded up to the alignment
        pl.chunk = chunk;
        layout(pl, a, p, own_w);
        if (pl.total <= budget) break;
      }
      if (chunk < m1) chunk -= chunk % kMinChunk;  // chunk starts stay 16-byte aligned in the split tables
      if (chunk < std::min(m1, kMinChunk)) continue;
    }
    pl.chunk = chunk;
    layout(pl, a, p, own_w);
    if (budget && pl.total > budget) continue;
    const int nchunks = (m1 + chunk - 1) / chunk;
    // (a ring that holds every block forms them in the first pass only, but the smaller
    // batches of more passes fill the sweep's point tiles worse: the model keeps one
    // recurrence per pass)
    const double cost = passes * (p->degree * spmm_bytes) + passes * (2.0 * nchunks - 1.0) * batch * e * es;
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = pl;
    }
    if (!budget || forced_passes) break;
    if (passes > 4096) break;
  }
  if (best_cost < 0) return fail(SSM_ERR_WORKSPACE, "no plan fits in %zu bytes of workspace", budget);
  out = best;
  return SSM_OK;
}

}  // namespace

struct ssm_ctx {
  ssm_csr a{};
  ssm_params p{};
  hipStream_t stream = nullptr;
  Plan pl;
  char* ws = nullptr;
  double* t = nullptr;
  double* c64 = nullptr;
  float* c32 = nullptr;
  __bf16* chi = nullptr;
  __bf16* clo = nullptr;
  int k3 = 0;  // split BF16: degrees k < k3 take three products, the rest one
  void* w = nullptr;
  void* y = nullptr;
  void* z = nullptr;
  char* ckpt = nullptr;  // checkpoint pairs (plan.ckpt > 0)
  double* kw = nullptr;
  double* kz = nullptr;
  double* gpart = nullptr;
  double* escr = nullptr;
  double* dos = nullptr;
  int32_t* ranks = nullptr;
  double* norm = nullptr;
  double* dpart = nullptr;  // DGC: workgroup partials of a group of steps
  double* dsums = nullptr;  // DGC: <Y_s, Y_s>, <Y_{s+1}, Y_s> per step
  double* dgc = nullptr;    // DGC: nt estimates, then M+1 moments
  // RESS-DGC
  double* nu = nullptr;     // (M+1) x ldc coefficients of the squared series
  double* kc = nullptr;     // nt x N~_v x N_v
  double* trw = nullptr;    // nt traces of K_W~
  double* hscr = nullptr;   // Algorithm 6 scratch
  double* pw = nullptr;     // S pair matrices (Y_{s+1}^T Y_s + Y_s^T Y_{s+1})/2
  double* pz = nullptr;     // S pair matrices Y_s^T Y_s
  double* xm = nullptr;     // moments X_0..X_M
  double* kmu = nullptr;    // nt x N_v'^2
  double* knu = nullptr;    // nt x N_v'^2
  double* xmax = nullptr;   // max |X_l[:N_v, :N_v]|, l <= M/2
  double* sfloor = nullptr; // rounding floor of Algorithm 4's truncation per point (null: none)
  double* mun = nullptr;    // SS-DGC: sqrt(sum_l mu_l(t_i)^2) per point
  double eta = 0.0;         // SS-DGC: scale of the rounding floor (0: no floor)
  ssm::RowOrder order;      // the recurrence's visiting order of the rows
  void* box = nullptr;      // A's values in box order (box stencils on the lattice), refreshed per call
  std::vector<double> dos_host;
  bool have_dos = false;
  bool have_dgc = false;
  ssm_stats stats{};
  std::vector<hipEvent_t> events;
  int last_batch_start = 0;
  bool z_valid = false;  // Z holds the last ssm_dos's blocks (the backward overwrites them)
  ssm_backward_stats bstats{};
};

extern "C" {

const char* ssm_last_error(void) { return g_last_error.c_str(); }

const char* ssm_status_str(ssm_status s) {
  switch (s) {
    case SSM_OK: return "ok";
    case SSM_ERR_ARG: return "invalid argument";
    case SSM_ERR_WORKSPACE: return "workspace too small or misaligned";
    case SSM_ERR_HIP: return "HIP runtime error";
    case SSM_ERR_BOUNDS: return "spectrum not inside [lo, hi]";
    case SSM_ERR_NONFINITE: return "non-finite value";
    case SSM_ERR_STATE: return "call order violated";
    case SSM_ERR_UNSUPPORTED: return "size not supported by this build";
  }
  return "unknown status";
}

ssm_status ssm_workspace_size(const ssm_csr* a, const ssm_params* p, size_t budget, size_t* bytes) {
  ssm_status s = check_csr(a);
  if (s != SSM_OK) return s;
  if ((s = check_params(p)) != SSM_OK) return s;
  if ((s = check_lattice(a, p)) != SSM_OK) return s;
  if (!bytes) return fail(SSM_ERR_ARG, "bytes is NULL");
  Plan pl;
  if ((s = make_plan(a, p, true, budget, pl)) != SSM_OK) return s;
  *bytes = pl.total;
  return SSM_OK;
}

ssm_status ssm_create(const ssm_csr* a, const ssm_params* p, const double* t_host, const void* w_dev,
                      void* workspace, size_t ws_bytes, void* stream, ssm_ctx** out) {
  ssm_status s = check_csr(a);
  if (s != SSM_OK) return s;
  if ((s = check_params(p)) != SSM_OK) return s;
  if ((s = check_lattice(a, p)) != SSM_OK) return s;
  if (!t_host || !out) return fail(SSM_ERR_ARG, "t_host and out must be non-NULL");
  for (int i = 0; i < p->nt; ++i)
    if (!std::isfinite(t_host[i])) return fail(SSM_ERR_ARG, "t[%d] is not finite", i);
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(SSM_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  const bool own_w = (w_dev == nullptr);
  Plan pl;
  if ((s = make_plan(a, p, own_w, ws_bytes, pl)) != SSM_OK) return s;
  if (pl.total > ws_bytes) return fail(SSM_ERR_WORKSPACE, "plan needs %zu bytes, got %zu", pl.total, ws_bytes);

  ssm_ctx* c = new ssm_ctx();
  c->a = *a;
  c->p = *p;
  c->p.tau = eff_tau(p);
  c->p.range_slack = eff_rho(p);
  c->stream = (hipStream_t)stream;
  c->pl = pl;
  c->ws = (char*)workspace;
  c->t = (double*)(c->ws + pl.off_t);
  c->c64 = (double*)(c->ws + pl.off_c64);
  // the FP32 copy of the table feeds the SS-DGC sweeps only (RESS-DGC sums moments in FP64)
  c->c32 = (p->precision == SSM_FP64 || pl.ress) ? nullptr : (float*)(c->ws + pl.off_c32);
  if (p->precision == SSM_FP32_BF16X3) {
    c->chi = (__bf16*)(c->ws + pl.off_chi);
    c->clo = (__bf16*)(c->ws + pl.off_clo);
  }
  c->w = own_w ? (void*)(c->ws + pl.off_w) : const_cast<void*>(w_dev);
  c->y = c->ws + pl.off_y;
  c->z = c->ws + pl.off_z;
  c->ckpt = pl.ckpt ? c->ws + pl.off_ckpt : nullptr;
  c->kw = (double*)(c->ws + pl.off_kw);
  c->kz = (double*)(c->ws + pl.off_kz);
  c->gpart = (double*)(c->ws + pl.off_gpart);
  c->escr = (double*)(c->ws + pl.off_escr);
  c->dos = (double*)(c->ws + pl.off_dos);
  c->ranks = (int32_t*)(c->ws + pl.off_ranks);
  c->norm = (double*)(c->ws + pl.off_norm);
  c->eta = eff_floor_scale(p);
  c->order = row_order(p);
  if (c->eta > 0) {
    c->mun = (double*)(c->ws + pl.off_mun);
    c->sfloor = (double*)(c->ws + pl.off_floor);
  }
  if (pl.dgc_group) {
    c->dpart = (double*)(c->ws + pl.off_dpart);
    c->dsums = (double*)(c->ws + pl.off_dsums);
    c->dgc = (double*)(c->ws + pl.off_dgc);
  }
  if (pl.ress) {
    c->z = nullptr;
    c->nu = (double*)(c->ws + pl.off_nu);
    c->kc = (double*)(c->ws + pl.off_kc);
    c->trw = (double*)(c->ws + pl.off_trw);
    c->hscr = (double*)(c->ws + pl.off_hscr);
    c->pw = (double*)(c->ws + pl.off_pw);
    c->pz = (double*)(c->ws + pl.off_pz);
    c->xm = (double*)(c->ws + pl.off_x);
    c->kmu = (double*)(c->ws + pl.off_kmu);
    c->knu = (double*)(c->ws + pl.off_knu);
    c->xmax = (double*)(c->ws + pl.off_xmax);
    c->sfloor = (double*)(c->ws + pl.off_floor);
  }
  c->dos_host.assign(p->nt, 0.0);

  auto bail = [&](ssm_status st) {
    delete c;
    return st;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(c->t, t_host, sizeof(double) * p->nt, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return bail(hip_fail(e, "copy of sweep points"));
  if (pl.ldc != p->nt) {  // padding columns of the coefficient table are read by the sweep: make them 0
    if ((e = hipMemsetAsync(c->c64, 0, (size_t)(p->degree + 1) * pl.ldc * 8, c->stream)) != hipSuccess)
      return bail(hip_fail(e, "clear coefficients"));
    if (c->c32 && (e = hipMemsetAsync(c->c32, 0, (size_t)(p->degree + 1) * pl.ldc * 4, c->stream)) != hipSuccess)
      return bail(hip_fail(e, "clear coefficients"));
  }
  const double c0 = 0.5 * (p->lo + p->hi), hw = 0.5 * (p->hi - p->lo);
  const double inv_norm = 1.0 / ((double)a->n * std::sqrt(2.0 * M_PI) * p->sigma);
  if ((e = ssm::launch_coefficients(c0, hw, p->sigma, inv_norm, c->t, p->nt, p->degree, n_theta_for(p->degree),
                                    c->c64, c->c32, pl.ldc, c->stream)) != hipSuccess)
    return bail(hip_fail(e, "coefficient kernel"));
  if (c->mun && (e = ssm::launch_coefficient_norms(c->c64, pl.ldc, p->nt, p->degree + 1, c->mun, c->stream)) !=
                    hipSuccess)
    return bail(hip_fail(e, "coefficient norm kernel"));
  if (c->chi) {
    if ((e = ssm::launch_split_blocks(c->c64, pl.ldc, p->nt, p->degree + 1, c->chi, c->clo, (int)(pl.ldk / 16), p->nt,
                                      c->stream)) != hipSuccess)
      return bail(hip_fail(e, "coefficient split kernel"));
  }
  if (pl.ress &&
      (e = ssm::launch_square_coefficients(c->c64, pl.ldc, p->nt, p->degree / 2, c->nu, pl.ldc, c->stream)) !=
          hipSuccess)
    return bail(hip_fail(e, "squared-series coefficient kernel"));
  if (own_w) {  // RESS-DGC: one block [W W~] of nv + nv_hybrid columns
    if ((e = ssm::launch_gaussian_block(p->seed, a->n, p->nv + p->nv_hybrid, p->precision == SSM_FP64 ? 0 : 1, c->w,
                                        c->stream)) != hipSuccess)
      return bail(hip_fail(e, "W generator"));
  }
  int box_bad = 1;
  if (pl.box_bytes) {  // is every row's pattern inside the 3 x 3 x 3 box of its point?
    int* flag = (int*)(c->ws + pl.off_box);
    if ((e = hipMemsetAsync(flag, 0, sizeof(int), c->stream)) != hipSuccess ||
        (e = ssm::launch_box_check(a->n, a->row_ptr, a->col_idx, p->lattice[0], p->lattice[1], p->lattice[2], flag,
                                   c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(&box_bad, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
      return bail(hip_fail(e, "box stencil check"));
  }
  std::vector<double> kmax;
  if (c->chi) {  // the largest coefficient of each degree
    kmax.resize(p->degree + 1);
    double* kmax_dev = (double*)(c->ws + pl.off_kmax);
    if ((e = ssm::launch_coefficient_row_max(c->c64, pl.ldc, p->nt, p->degree + 1, kmax_dev, c->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(kmax.data(), kmax_dev, kmax.size() * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream)) != hipSuccess)
      return bail(hip_fail(e, "largest coefficient per degree"));
  }
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(hip_fail(e, "ssm_create sync"));
  if (c->chi) c->k3 = three_product_degrees(kmax);
  if (pl.box_bytes && !box_bad) {
    c->box = c->ws + pl.off_box;
    c->order.box = c->box;
    c->stats.box_stencil = 1;
  }
  c->stats.passes = pl.passes;
  c->stats.chunk = pl.chunk;
  c->stats.batch = pl.batch;
  c->stats.gram_segments = pl.nseg;
  c->stats.split_k3 = c->k3;
  if (pl.ress) c->stats.chunk = pl.chunk + 1;  // ring slots
  *out = c;
  return SSM_OK;
}

ssm_status ssm_destroy(ssm_ctx* c) {
  if (!c) return fail(SSM_ERR_ARG, "ctx is NULL");
  for (auto ev : c->events) (void)hipEventDestroy(ev);
  delete c;
  return SSM_OK;
}

namespace {
ssm_status ress_dos(ssm_ctx* c, double* dos_host, int32_t* ranks_host);

// A's values in box order, from the CSR as it is now (the values may change between calls)
ssm_status refresh_box(ssm_ctx* c) {
  if (!c->box) return SSM_OK;
  const int32_t* lt = c->p.lattice;
  hipError_t e = ssm::launch_box_values(c->a.n, c->a.row_ptr, c->a.col_idx, c->a.values, c->p.precision != SSM_FP64,
                                        lt[0], lt[1], lt[2], c->box, c->stream);
  return e == hipSuccess ? SSM_OK : hip_fail(e, "box values");
}
}

namespace {

struct Span { size_t b, en; int kind; };  // kind 0 recurrence, 1 sweep, 2 Gram, 3 Algorithm 4

// Event bookkeeping of one ssm_dos (the context's events, recorded in order).
struct Timeline {
  size_t next = 0;
  std::vector<Span> spans;
  size_t mark() { return next++; }
};

// One pass of Algorithm 5 over sweep-point batch `pass`: the recurrence (steps 3, 9-10)
// chunk by chunk into the ring, each chunk followed by its sweep (steps 6-8) into the
// batch's Z.  A plan whose ring holds every block forms the blocks in its first pass only.
// `first`: the first pass of an ssm_dos, which also keeps the checkpoint pairs and the
// inner products of Algorithm 2.  The backward calls it again to regenerate a batch's Z:
// the same launches in the same order, so the blocks and Z are bit-identical to the
// forward's.  tl (may be null) records the recurrence and sweep spans.
ssm_status forward_pass(ssm_ctx* c, int pass, bool first, Timeline* tl, int64_t& spmm_launches,
                        int64_t& sweep_launches) {
  const ssm_params& p = c->p;
  const Plan& pl = c->pl;
  const int64_t n = c->a.n;
  const int nv = p.nv;
  const int64_t e = n * nv;
  const size_t es = elem_bytes(p.precision);
  const bool f64 = p.precision == SSM_FP64;
  const double alpha = 2.0 / (p.hi - p.lo);
  const double beta = -(p.hi + p.lo) / (p.hi - p.lo);
  const int m = p.degree;
  hipStream_t st = c->stream;
  const int nchunks = (m + 1 + pl.chunk - 1) / pl.chunk;
  const bool resident = pl.chunk == m + 1;
  auto y_slot = [&](int k) -> char* { return (char*)c->y + (size_t)(k % pl.chunk) * e * es; };
  auto record = [&](size_t i) { return tl ? hipEventRecord(c->events[i], st) : hipSuccess; };
  const int64_t dgc_nblocks = ssm::cheb_step_blocks(n, nv, !f64);
  const int p0 = pass * pl.batch;
  const int nb = std::min(pl.batch, p.nt - p0);
  for (int ch = 0; ch < nchunks; ++ch) {
    const int k_first = ch * pl.chunk;
    const int k_last = std::min(m, k_first + pl.chunk - 1);
    if (!resident || pass == 0) {
      Span rs{tl ? tl->mark() : 0, 0, 0};
      SSM_HIP(record(rs.b), "hipEventRecord");
      for (int k = k_first; k <= k_last; ++k) {
        char* out = y_slot(k);
        hipError_t err;
        if (k == 0) {
          err = hipMemcpyAsync(out, c->w, e * es, hipMemcpyDeviceToDevice, st);
        } else {
          const void* x = (k == 1) ? c->w : (const void*)y_slot(k - 1);
          const void* xp = (k == 1) ? nullptr : (const void*)y_slot(k - 2);
          const double a = (k == 1) ? alpha : 2.0 * alpha;
          const double b = (k == 1) ? beta : 2.0 * beta;
          const double cc = (k == 1) ? 0.0 : -1.0;
          const int s_step = k - 1;  // this step forms Y_{s+1} from Y_s
          const bool moments = first && pl.dgc_group && s_step < dgc_steps(m);
          double* dots = moments ? c->dpart + (size_t)(s_step % pl.dgc_group) * 2 * dgc_nblocks : nullptr;
          if (f64)
            err = ssm::launch_cheb_step_f64(n, nv, c->a.row_ptr, c->a.col_idx, (const double*)c->a.values, a, b, cc,
                                            (const double*)x, (const double*)xp, nullptr, (double*)out, st, dots,
                                            c->order);
          else
            err = ssm::launch_cheb_step_f32(n, nv, c->a.row_ptr, c->a.col_idx, (const float*)c->a.values, (float)a,
                                            (float)b, (float)cc, (const float*)x, (const float*)xp, nullptr,
                                            (float*)out, st, dots, c->order);
          ++spmm_launches;
          if (err == hipSuccess && moments &&
              (s_step % pl.dgc_group == pl.dgc_group - 1 || s_step == dgc_steps(m) - 1)) {
            const int s0 = s_step - s_step % pl.dgc_group;
            err = ssm::launch_moments(dgc_nblocks, c->dpart, s0, s_step - s0 + 1, c->dsums, st);
          }
        }
        if (err != hipSuccess) return hip_fail(err, "Chebyshev step");
        if (pl.ckpt && first) {  // keep the checkpoint pairs for the adjoint
          const int j = (k + 1) / pl.ckpt;
          const int cf = ckpt_first(j, pl.ckpt);
          if ((k == cf || k == cf + 1) && j < ckpt_pairs(m, pl.ckpt)) {
            err = hipMemcpyAsync(c->ckpt + (size_t)(2 * j + (k - cf)) * e * es, out, e * es,
                                 hipMemcpyDeviceToDevice, st);
            if (err != hipSuccess) return hip_fail(err, "checkpoint copy");
          }
        }
      }
      rs.en = tl ? tl->mark() : 0;
      SSM_HIP(record(rs.en), "hipEventRecord");
      if (tl) tl->spans.push_back(rs);
    }
    // sweep over this chunk
    Span ss{tl ? tl->mark() : 0, 0, 1};
    SSM_HIP(record(ss.b), "hipEventRecord");
    const int kc = k_last - k_first + 1;
    hipError_t err;
    if (f64)
      err = ssm::launch_sweep_f64(e, kc, nb, c->c64 + (int64_t)k_first * pl.ldc + p0, pl.ldc, pl.ldc - p0,
                                  (const double*)y_slot(k_first), (double*)c->z, ch > 0, st);
    else if (p.precision == SSM_FP32_BF16X3) {
      // the split tables are in 16-degree blocks of nt rows; chunk starts are multiples of 16
      if (k_first % 16) return fail(SSM_ERR_STATE, "ring chunk starts at degree %d, not a multiple of 16", k_first);
      const int64_t off = ((int64_t)(k_first / 16) * p.nt + p0) * 16;
      err = ssm::launch_sweep_bf16x3(e, kc, nb, c->chi + off, c->clo + off, 16, p.nt - p0,
                                     (int64_t)p.nt * pl.ldk - off, (const float*)y_slot(k_first), (float*)c->z,
                                     ch > 0, c->k3 - k_first, nb, st, (int64_t)16 * p.nt);
    } else if (p.precision == SSM_FP32)
      err = ssm::launch_sweep_f32(e, kc, nb, c->c32 + (int64_t)k_first * pl.ldc + p0, pl.ldc, pl.ldc - p0,
                                  (const float*)y_slot(k_first), (float*)c->z, ch > 0, st);
    else
      err = ssm::launch_sweep_bf16(e, kc, nb, c->c32 + (int64_t)k_first * pl.ldc + p0, pl.ldc, pl.ldc - p0,
                                   (const float*)y_slot(k_first), (float*)c->z, ch > 0, st);
    if (err != hipSuccess) return hip_fail(err, "sweep GEMM");
    ++sweep_launches;
    ss.en = tl ? tl->mark() : 0;
    SSM_HIP(record(ss.en), "hipEventRecord");
    if (tl) tl->spans.push_back(ss);
  }
  return SSM_OK;
}

}  // namespace

ssm_status ssm_dos(ssm_ctx* c, double* dos_host, int32_t* ranks_host) {
  if (!c || !dos_host) return fail(SSM_ERR_ARG, "ctx and dos_host must be non-NULL");
  ssm_status bs = refresh_box(c);
  if (bs != SSM_OK) return bs;
  if (c->pl.ress) return ress_dos(c, dos_host, ranks_host);
  const ssm_params& p = c->p;
  const Plan& pl = c->pl;
  const int64_t n = c->a.n;
  const int nv = p.nv;
  const int64_t e = n * nv;
  const size_t es = elem_bytes(p.precision);
  const bool f64 = p.precision == SSM_FP64;
  const int m = p.degree;
  hipStream_t st = c->stream;

  // events: [0] start, then (begin, end) pairs per timed launch group
  const int nchunks = (m + 1 + pl.chunk - 1) / pl.chunk;
  const size_t need = 2 + (size_t)pl.passes * (2 * nchunks + 2) * 2 + 4;
  while (c->events.size() < need) {
    hipEvent_t ev;
    SSM_HIP(hipEventCreate(&ev), "hipEventCreate");
    c->events.push_back(ev);
  }
  Timeline tl;
  auto mark = [&]() -> size_t { return tl.mark(); };
  const size_t ev_start = mark();
  SSM_HIP(hipEventRecord(c->events[ev_start], st), "hipEventRecord");
  int64_t spmm_launches = 0, sweep_launches = 0;
  c->z_valid = false;

  auto y_slot = [&](int k) -> char* { return (char*)c->y + (size_t)(k % pl.chunk) * e * es; };
  const double g_max = 1.0 / ((double)n * std::sqrt(2.0 * M_PI) * p.sigma);
  for (int pass = 0; pass < pl.passes; ++pass) {
    const int p0 = pass * pl.batch;
    const int nb = std::min(pl.batch, p.nt - p0);
    ssm_status fs = forward_pass(c, pass, pass == 0, &tl, spmm_launches, sweep_launches);
    if (fs != SSM_OK) return fs;
    if (pass == 0) {  // bound check inputs: ||W||_F^2 and ||T_M(A~) W||_F^2
      hipError_t err = ssm::launch_sumsq(c->w, e, !f64, c->norm + 8, c->norm + 0, st);
      if (err == hipSuccess) err = ssm::launch_sumsq(y_slot(m), e, !f64, c->norm + 8, c->norm + 1, st);
      if (err == hipSuccess && c->sfloor)  // eta ||mu(t_i)||_2 ||W||_F^2 / sqrt(N N_v)
        err = ssm::launch_rounding_floor(c->mun, p.nt, c->eta, c->norm + 0, 1.0 / std::sqrt((double)e), c->sfloor, st);
      if (err != hipSuccess) return hip_fail(err, "norm kernel");
    }
    Span gs{mark(), mark(), 2};
    SSM_HIP(hipEventRecord(c->events[gs.b], st), "hipEventRecord");
    hipError_t err = ssm::launch_gram(!f64, n, nv, nb, c->w, c->z, c->kw + (int64_t)p0 * nv * nv,
                                      c->kz + (int64_t)p0 * nv * nv, pl.nseg, c->gpart, st);
    if (err != hipSuccess) return hip_fail(err, "Gram kernel");
    SSM_HIP(hipEventRecord(c->events[gs.en], st), "hipEventRecord");
    tl.spans.push_back(gs);
    c->last_batch_start = p0;
  }
  Span es_{mark(), mark(), 3};
  SSM_HIP(hipEventRecord(c->events[es_.b], st), "hipEventRecord");
  hipError_t err = ssm::launch_geneig_trace(nv, p.nt, c->kw, c->kz, g_max, p.tau, p.range_slack, c->dos, c->ranks,
                                            c->escr, st, 0, nullptr, nullptr, nullptr, c->sfloor);
  if (err != hipSuccess) return hip_fail(err, "Algorithm 4 kernel");
  SSM_HIP(hipEventRecord(c->events[es_.en], st), "hipEventRecord");
  tl.spans.push_back(es_);
  if (pl.dgc_group) {
    err = ssm::launch_dgc(c->c64, pl.ldc, p.nt, m + 1, nv, c->dsums, c->dgc, c->dgc + p.nt, st);
    if (err != hipSuccess) return hip_fail(err, "Algorithm 2 kernel");
  }

  std::vector<double> dos(p.nt);
  std::vector<int32_t> ranks(2 * (size_t)p.nt);
  double norms[2];
  SSM_HIP(hipMemcpyAsync(dos.data(), c->dos, sizeof(double) * p.nt, hipMemcpyDeviceToHost, st), "copy DOS");
  SSM_HIP(hipMemcpyAsync(ranks.data(), c->ranks, sizeof(int32_t) * 2 * p.nt, hipMemcpyDeviceToHost, st), "copy ranks");
  SSM_HIP(hipMemcpyAsync(norms, c->norm, sizeof(norms), hipMemcpyDeviceToHost, st), "copy norms");
  SSM_HIP(hipStreamSynchronize(st), "ssm_dos sync");

  ssm_stats& S = c->stats;
  S.ms_recurrence = S.ms_sweep = S.ms_gram = S.ms_geneig = 0.0;
  for (const Span& sp : tl.spans) {
    float ms = 0.f;
    SSM_HIP(hipEventElapsedTime(&ms, c->events[sp.b], c->events[sp.en]), "hipEventElapsedTime");
    double* dst = sp.kind == 0 ? &S.ms_recurrence : sp.kind == 1 ? &S.ms_sweep : sp.kind == 2 ? &S.ms_gram : &S.ms_geneig;
    *dst += ms;
  }
  float tot = 0.f;
  SSM_HIP(hipEventElapsedTime(&tot, c->events[ev_start], c->events[es_.en]), "hipEventElapsedTime");
  S.ms_total = tot;
  S.spmm_launches = spmm_launches;
  S.sweep_launches = sweep_launches;

  if (std::isnan(norms[0]) || std::isnan(norms[1]))
    return fail(SSM_ERR_NONFINITE, "NaN in W or T_M(A~)W: non-finite values, or [lo, hi] far from enclosing spec(A)");
  if (!std::isfinite(norms[0]) || !std::isfinite(norms[1]) || norms[1] > (1.0 + 1e-3) * (1.0 + 1e-3) * norms[0])
    return fail(SSM_ERR_BOUNDS, "||T_M(A~)W||_F^2 = %g exceeds ||W||_F^2 = %g: spectrum not inside [lo, hi]",
                norms[1], norms[0]);
  for (int i = 0; i < p.nt; ++i)
    if (!std::isfinite(dos[i])) return fail(SSM_ERR_NONFINITE, "DOS at point %d is not finite", i);
  std::copy(dos.begin(), dos.end(), dos_host);
  if (ranks_host) std::copy(ranks.begin(), ranks.end(), ranks_host);
  c->dos_host = dos;
  c->have_dos = true;
  c->have_dgc = pl.dgc_group > 0;
  c->z_valid = true;
  return SSM_OK;
}

// ---------------------------------------------------------------------------
// RESS-DGC driver (Algorithm 7, Theorem 4)
// ---------------------------------------------------------------------------
namespace {

// Algorithm 4's truncation under RESS-DGC also drops eigenvalues of K_W below
// kRessFloor * sum_{l<=M/2} |mu_l(t_i)| max|X_l|: the rounding level of K_W formed as a
// sum of moments (about 4500 units of FP64 rounding).  Without it, at sweep points where
// g^{M/2}(t_i I - A) W is rounding noise, K_Z's independent rounding gives the pencil
// arbitrary eigenvalues, in range included.
constexpr double kRessFloor = 1e-12;
// With an FP32 recurrence the moments carry the blocks' rounding, which grows with the
// degree and is doubled by the product identity: the floor is 2^-18 of the same sum, about
// 32 units of FP32 rounding (a host model of the FP32 moments on the 32 x 32 workload gave
// DOS L1 errors against FP64 of 1.4e-2, 2.2e-4 and 7e-6 with 1e-12, 2^-22 and 2^-18).
constexpr double kRessFloorF32 = 0x1p-18;

ssm_status ress_dos(ssm_ctx* c, double* dos_host, int32_t* ranks_host) {
  const ssm_params& p = c->p;
  const Plan& pl = c->pl;
  const int64_t n = c->a.n;
  const int nv = p.nv, nvh = p.nv_hybrid, nvp = nv + nvh;
  const int64_t e = n * nvp;
  const int64_t nnp = (int64_t)nvp * nvp;
  const int m = p.degree, m1 = m + 1;
  const int S = m / 2 + 1;          // pairs (Y_s, Y_{s+1}), s = 0..M/2
  const int R = pl.chunk + 1;       // ring slots
  const double alpha = 2.0 / (p.hi - p.lo);
  const double beta = -(p.hi + p.lo) / (p.hi - p.lo);
  const bool f64 = p.precision == SSM_FP64;
  const size_t es = elem_bytes(p.precision);
  hipStream_t st = c->stream;
  const int rounds = (S + pl.chunk - 1) / pl.chunk;
  const size_t need = 4 * (size_t)rounds + 8;
  while (c->events.size() < need) {
    hipEvent_t ev;
    SSM_HIP(hipEventCreate(&ev), "hipEventCreate");
    c->events.push_back(ev);
  }
  size_t evi = 0;
  struct Span { size_t b, en; int kind; };  // 0 rec, 1 moments + per-point sums, 2 pair Gram, 3 eig
  std::vector<Span> spans;
  auto mark = [&]() -> size_t { return evi++; };
  auto rec = [&](size_t ev) { return hipEventRecord(c->events[ev], st); };
  const size_t ev_start = mark();
  SSM_HIP(rec(ev_start), "hipEventRecord");
  auto slot = [&](int k) -> char* { return (char*)c->y + (size_t)(k % R) * e * es; };
  int64_t spmm_launches = 0;
  hipError_t err = hipMemcpyAsync(slot(0), c->w, e * es, hipMemcpyDeviceToDevice, st);
  if (err != hipSuccess) return hip_fail(err, "copy of W");
  int k = 0;       // last block formed
  int s_done = 0;  // next pair to form
  while (s_done < S) {
    // a round forms Y_{k+1}..Y_{k_last}; the ring (chunk + 1 slots) still holds Y_{s_done}
    const int k_last = std::min(S, s_done + pl.chunk);
    Span rs{mark(), 0, 0};
    SSM_HIP(rec(rs.b), "hipEventRecord");
    for (int kk = k + 1; kk <= k_last; ++kk) {
      const char* x = slot(kk - 1);
      const char* xp = kk == 1 ? nullptr : slot(kk - 2);
      const double sa = kk == 1 ? alpha : 2.0 * alpha, sb = kk == 1 ? beta : 2.0 * beta, sc = kk == 1 ? 0.0 : -1.0;
      if (f64)
        err = ssm::launch_cheb_step_f64(n, nvp, c->a.row_ptr, c->a.col_idx, (const double*)c->a.values, sa, sb, sc,
                                        (const double*)x, (const double*)xp, nullptr, (double*)slot(kk), st, nullptr,
                                        c->order);
      else
        err = ssm::launch_cheb_step_f32(n, nvp, c->a.row_ptr, c->a.col_idx, (const float*)c->a.values, (float)sa,
                                        (float)sb, (float)sc, (const float*)x, (const float*)xp, nullptr,
                                        (float*)slot(kk), st, nullptr, c->order);
      if (err != hipSuccess) return hip_fail(err, "Chebyshev step");
      ++spmm_launches;
    }
    k = k_last;
    rs.en = mark();
    SSM_HIP(rec(rs.en), "hipEventRecord");
    spans.push_back(rs);
    // pairs s_done..k_last-1, in runs whose two slots do not wrap
    Span gs{rs.en, 0, 2};
    for (int a = s_done; a < k_last;) {
      const int sa = a % R;
      const int len = sa == R - 1 ? 1 : std::min(k_last - a, R - 1 - sa);
      const char* lo_blk = (const char*)c->y + (size_t)sa * e * es;
      const char* hi_blk = sa == R - 1 ? (const char*)c->y : lo_blk + e * es;
      err = ssm::launch_gram_pairs(!f64, n, nvp, len, hi_blk, lo_blk, e, c->pw + (int64_t)a * nnp,
                                   c->pz + (int64_t)a * nnp, pl.nseg, c->gpart, st);
      if (err != hipSuccess) return hip_fail(err, "pair Gram kernel");
      a += len;
    }
    gs.en = mark();
    SSM_HIP(rec(gs.en), "hipEventRecord");
    spans.push_back(gs);
    s_done = k_last;
  }
  // bound check inputs: ||V||_F^2 and ||T_{M/2+1}(A~) V||_F^2
  err = ssm::launch_sumsq(c->w, e, !f64, c->norm + 8, c->norm + 0, st);
  if (err == hipSuccess) err = ssm::launch_sumsq(slot(S), e, !f64, c->norm + 8, c->norm + 1, st);
  if (err != hipSuccess) return hip_fail(err, "norm kernel");
  // moments and the per-point sums (FP64 sweep GEMM over X, blocks of N_v'^2 entries)
  Span ms{mark(), 0, 1};
  SSM_HIP(rec(ms.b), "hipEventRecord");
  err = ssm::launch_ress_moments(nvp, m1, c->pw, c->pz, c->xm, st);
  if (err == hipSuccess)
    err = ssm::launch_sweep_f64(nnp, S, p.nt, c->c64, pl.ldc, pl.ldc, c->xm, c->kmu, 0, st);
  if (err == hipSuccess)
    err = ssm::launch_sweep_f64(nnp, m1, p.nt, c->nu, pl.ldc, pl.ldc, c->xm, c->knu, 0, st);
  if (err == hipSuccess) err = ssm::launch_ress_extract(p.nt, nv, nvh, c->kmu, c->knu, c->kw, c->kz, c->kc, c->trw, st);
  if (err == hipSuccess)
    err = ssm::launch_ress_floor(nv, nvp, m / 2, c->xm, c->c64, pl.ldc, p.nt, f64 ? kRessFloor : kRessFloorF32,
                                 c->xmax, c->sfloor, st);
  if (err != hipSuccess) return hip_fail(err, "moment kernels");
  ms.en = mark();
  SSM_HIP(rec(ms.en), "hipEventRecord");
  spans.push_back(ms);
  const double g_max = 1.0 / ((double)n * std::sqrt(2.0 * M_PI) * p.sigma);
  Span es_{mark(), mark(), 3};
  SSM_HIP(rec(es_.b), "hipEventRecord");
  err = ssm::launch_geneig_trace(nv, p.nt, c->kw, c->kz, g_max, p.tau, p.range_slack, c->dos, c->ranks, c->escr, st,
                                 nvh, c->kc, c->trw, c->hscr, c->sfloor);
  if (err != hipSuccess) return hip_fail(err, "Algorithm 4 kernel");
  SSM_HIP(rec(es_.en), "hipEventRecord");
  spans.push_back(es_);

  std::vector<double> dos(p.nt);
  std::vector<int32_t> ranks(2 * (size_t)p.nt);
  double norms[2];
  SSM_HIP(hipMemcpyAsync(dos.data(), c->dos, sizeof(double) * p.nt, hipMemcpyDeviceToHost, st), "copy DOS");
  SSM_HIP(hipMemcpyAsync(ranks.data(), c->ranks, sizeof(int32_t) * 2 * p.nt, hipMemcpyDeviceToHost, st), "copy ranks");
  SSM_HIP(hipMemcpyAsync(norms, c->norm, sizeof(norms), hipMemcpyDeviceToHost, st), "copy norms");
  SSM_HIP(hipStreamSynchronize(st), "ssm_dos sync");
  ssm_stats& Sx = c->stats;
  Sx.ms_recurrence = Sx.ms_sweep = Sx.ms_gram = Sx.ms_geneig = 0.0;
  for (const Span& sp : spans) {
    float ms_ = 0.f;
    SSM_HIP(hipEventElapsedTime(&ms_, c->events[sp.b], c->events[sp.en]), "hipEventElapsedTime");
    double* dst = sp.kind == 0 ? &Sx.ms_recurrence : sp.kind == 1 ? &Sx.ms_sweep : sp.kind == 2 ? &Sx.ms_gram
                                                                                    : &Sx.ms_geneig;
    *dst += ms_;
  }
  float tot = 0.f;
  SSM_HIP(hipEventElapsedTime(&tot, c->events[ev_start], c->events[es_.en]), "hipEventElapsedTime");
  Sx.ms_total = tot;
  Sx.spmm_launches = spmm_launches;
  Sx.sweep_launches = 2;
  if (std::isnan(norms[0]) || std::isnan(norms[1]))
    return fail(SSM_ERR_NONFINITE, "NaN in W or T_{M/2+1}(A~)W: non-finite values, or [lo, hi] far from spec(A)");
  if (!std::isfinite(norms[0]) || !std::isfinite(norms[1]) || norms[1] > (1.0 + 1e-3) * (1.0 + 1e-3) * norms[0])
    return fail(SSM_ERR_BOUNDS, "||T_{M/2+1}(A~)W||_F^2 = %g exceeds ||W||_F^2 = %g: spectrum not inside [lo, hi]",
                norms[1], norms[0]);
  for (int i = 0; i < p.nt; ++i)
    if (!std::isfinite(dos[i])) return fail(SSM_ERR_NONFINITE, "DOS at point %d is not finite", i);
  std::copy(dos.begin(), dos.end(), dos_host);
  if (ranks_host) std::copy(ranks.begin(), ranks.end(), ranks_host);
  c->dos_host = dos;
  c->have_dos = true;
  c->z_valid = false;
  return SSM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------
namespace {

constexpr int kBackwardSegment = 256;  // Ybar blocks formed per transposed-sweep launch (resident blocks)

// How the backward walks the degrees.  Level-1 segments are [j S, min((j+1) S - 1, M)] for
// the forward's checkpoint interval S (one segment [0, M] when every block is resident).
// Each is cut into sub-segments of at most `sub` reverse steps, top first; a sub-segment's
// blocks T_{k-1}(A~)W come from the resident ring, or are recomputed into the ring from the
// pair (Y_{b0}, Y_{b0+1}), b0 = first degree - 1: the level-1 checkpoint pair for a
// segment's first sub-segment, else a level-2 pair that a replay of the segment from its
// level-1 pair left in the backward workspace (two levels when the ring holds fewer than
// S blocks).
struct BackwardLayout {
  size_t phibar, kwb, kzb, gescr, ct64, ct32, chit, clot, lam, ybar, pairs2, total;
  int64_t ldct, ldkt;
  int sub;      // reverse steps per sub-segment (and Ybar blocks per transposed sweep, + 3)
  int levels;   // 0: blocks resident; 1: checkpoints, segment recomputed into the ring; 2: two levels
  int npairs2;  // level-2 pairs per level-1 segment
};

BackwardLayout backward_layout(const ssm_ctx* c) {
  const ssm_params& p = c->p;
  const Plan& pl = c->pl;
  const size_t es = elem_bytes(p.precision);
  const size_t e = (size_t)c->a.n * p.nv;
  const size_t nn = (size_t)p.nv * p.nv;
  const int m1 = p.degree + 1;
  BackwardLayout L{};
  L.ldct = (m1 + 3) / 4 * 4;
  L.ldkt = (p.nt + 63) / 64 * 64;  // 128-byte rows, as the forward tables
  if (!pl.ckpt) {
    L.levels = 0;
    L.sub = std::min(kBackwardSegment, m1);
  } else if (pl.chunk >= pl.ckpt) {
    L.levels = 1;
    L.sub = pl.ckpt;
  } else {
    L.levels = 2;
    L.sub = pl.chunk;
    L.npairs2 = (pl.ckpt + L.sub - 1) / L.sub;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += align_up(bytes);
    return r;
  };
  L.phibar = take(p.nt * 8);
  L.kwb = take(p.nt * nn * 8);
  L.kzb = take(p.nt * nn * 8);
  L.gescr = take((size_t)ssm::geneig_backward_scratch_total(p.nv, p.nt) * 8);
  L.ct64 = take(p.precision == SSM_FP64 ? (size_t)p.nt * L.ldct * 8 : 0);
  L.ct32 = take(p.precision == SSM_FP32 || p.precision == SSM_FP32_BF16SWEEP ? (size_t)p.nt * L.ldct * 4 : 0);
  L.chit = take(p.precision == SSM_FP32_BF16X3 ? (size_t)m1 * L.ldkt * 2 : 0);
  L.clot = take(p.precision == SSM_FP32_BF16X3 ? (size_t)m1 * L.ldkt * 2 : 0);
  L.lam = take(3 * e * es);
  L.ybar = take((size_t)(L.sub + 3) * e * es);  // + 3: a sub-segment's rows start at a multiple of 4
  L.pairs2 = take((size_t)2 * L.npairs2 * e * es);
  L.total = o;
  return L;
}

}  // namespace

ssm_status ssm_backward_workspace_size(const ssm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(SSM_ERR_ARG, "ctx and bytes must be non-NULL");
  *bytes = backward_layout(c).total;
  return SSM_OK;
}

ssm_status ssm_get_backward_stats(const ssm_ctx* c, ssm_backward_stats* out) {
  if (!c || !out) return fail(SSM_ERR_ARG, "ctx and out must be non-NULL");
  *out = c->bstats;
  return SSM_OK;
}

ssm_status ssm_backward(ssm_ctx* c, const double* dos_bar_host, double* grad_dev, void* workspace, size_t ws_bytes) {
  if (!c || !dos_bar_host || !grad_dev || !workspace) return fail(SSM_ERR_ARG, "pointers must be non-NULL");
  const ssm_params& p = c->p;
  const Plan& pl = c->pl;
  const int m = p.degree, m1 = m + 1;
  if (pl.ress) return fail(SSM_ERR_UNSUPPORTED, "no adjoint for RESS-DGC in this build");
  if (pl.chunk != m1 && !pl.ckpt)
    return fail(SSM_ERR_UNSUPPORTED,
                "the adjoint needs a plan whose ring holds every T_k(A~)W, or one made with ckpt_every > 0");
  if (!c->have_dos) return fail(SSM_ERR_STATE, "ssm_backward needs a preceding ssm_dos");
  for (int i = 0; i < p.nt; ++i)
    if (!std::isfinite(dos_bar_host[i])) return fail(SSM_ERR_ARG, "dos_bar[%d] is not finite", i);
  ssm_status bs = refresh_box(c);  // blocks formed again here take A's values as they are now
  if (bs != SSM_OK) return bs;
  const BackwardLayout L = backward_layout(c);
  if (ws_bytes < L.total || ((uintptr_t)workspace % kAlign))
    return fail(SSM_ERR_WORKSPACE, "backward needs %zu bytes (256-byte aligned), got %zu", L.total, ws_bytes);
  char* ws = (char*)workspace;
  const int64_t n = c->a.n;
  const int nv = p.nv;
  const int64_t e = n * nv;
  const int64_t nn = (int64_t)nv * nv;
  const size_t es = elem_bytes(p.precision);
  const size_t bb = (size_t)e * es;  // bytes per block
  const bool f64 = p.precision == SSM_FP64;
  const double alpha = 2.0 / (p.hi - p.lo);
  const double beta = -(p.hi + p.lo) / (p.hi - p.lo);
  const double g_max = 1.0 / ((double)n * std::sqrt(2.0 * M_PI) * p.sigma);
  hipStream_t st = c->stream;
  double* phibar = (double*)(ws + L.phibar);
  double* kwb = (double*)(ws + L.kwb);
  double* kzb = (double*)(ws + L.kzb);
  double* gescr = (double*)(ws + L.gescr);
  char* lam = ws + L.lam;
  char* ybar = ws + L.ybar;
  char* pairs2 = ws + L.pairs2;
  char* ring = (char*)c->y;
  auto lam_slot = [&](int k) { return lam + (size_t)(k % 3) * bb; };
  // Y_{b} from Y_{b-1} (x) and Y_{b-2} (xp): b = 1 takes a = alpha, b = beta, no xp
  auto cheb = [&](const void* x, const void* xp, void* out) {
    const double a = xp ? 2 * alpha : alpha, b = xp ? 2 * beta : beta, cc = xp ? -1.0 : 0.0;
    if (f64)
      return ssm::launch_cheb_step_f64(n, nv, c->a.row_ptr, c->a.col_idx, (const double*)c->a.values, a, b, cc,
                                       (const double*)x, (const double*)xp, nullptr, (double*)out, st, nullptr,
                                       c->order);
    return ssm::launch_cheb_step_f32(n, nv, c->a.row_ptr, c->a.col_idx, (const float*)c->a.values, (float)a,
                                     (float)b, (float)cc, (const float*)x, (const float*)xp, nullptr, (float*)out, st,
                                     nullptr, c->order);
  };

  hipEvent_t ev[2] = {};
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  for (auto& x : ev) SSM_HIP(hipEventCreate(&x), "hipEventCreate");
  // time of the launches enqueued by f, on the stream (synchronises)
  auto timed = [&](float& acc, auto f) -> ssm_status {
    SSM_HIP(hipEventRecord(ev[0], st), "hipEventRecord");
    ssm_status s2 = f();
    if (s2 != SSM_OK) return s2;
    SSM_HIP(hipEventRecord(ev[1], st), "hipEventRecord");
    SSM_HIP(hipEventSynchronize(ev[1]), "hipEventSynchronize");
    float t = 0.f;
    SSM_HIP(hipEventElapsedTime(&t, ev[0], ev[1]), "hipEventElapsedTime");
    acc += t;
    return SSM_OK;
  };
  float ms_ge = 0.f, ms_zb = 0.f, ms_ybar = 0.f, ms_rc = 0.f, ms_rev = 0.f, ms_fwd = 0.f;
  int recomputed = 0, subsegs = 0;
  ssm_status s0;

  // Algorithm 4 backward for every sweep point (K_W, K_Z of all batches are kept), the
  // transposed coefficient tables for Ybar = C Zbar, and the gradient cleared
  s0 = timed(ms_ge, [&]() -> ssm_status {
    SSM_HIP(hipMemcpyAsync(phibar, dos_bar_host, sizeof(double) * p.nt, hipMemcpyHostToDevice, st), "copy dos_bar");
    hipError_t err = ssm::launch_geneig_backward(nv, p.nt, c->kw, c->kz, g_max, p.tau, p.range_slack, phibar, kwb,
                                                 kzb, gescr, st, c->sfloor);
    if (err != hipSuccess) return hip_fail(err, "Algorithm 4 backward kernel");
    if (p.precision == SSM_FP32_BF16X3)
      err = ssm::launch_split_rows(c->c64, pl.ldc, p.nt, m1, (__bf16*)(ws + L.chit), (__bf16*)(ws + L.clot), L.ldkt,
                                   st);
    else
      err = ssm::launch_transpose_coefficients(c->c64, pl.ldc, p.nt, m1, f64 ? (double*)(ws + L.ct64) : nullptr,
                                               f64 ? nullptr : (float*)(ws + L.ct32), L.ldct, st);
    if (err != hipSuccess) return hip_fail(err, "adjoint set-up kernels");
    SSM_HIP(hipMemsetAsync(grad_dev, 0, sizeof(double) * c->a.nnz, st), "clear gradient");
    return SSM_OK;
  });
  if (s0 != SSM_OK) return s0;

  // the batches: the one whose Z the last ssm_dos left resident first, then the others
  // with Z regenerated by the forward pass
  const int resident_pass = c->last_batch_start / pl.batch;
  for (int bi = 0; bi < pl.passes; ++bi) {
    const int pass = bi == 0 ? resident_pass : (bi - 1 < resident_pass ? bi - 1 : bi);
    const int p0 = pass * pl.batch;
    const int nb = std::min(pl.batch, p.nt - p0);
    if (bi > 0 || !c->z_valid) {
      int64_t n_spmm = 0, n_sweep = 0;
      s0 = timed(ms_fwd, [&]() { return forward_pass(c, pass, false, nullptr, n_spmm, n_sweep); });
      if (s0 != SSM_OK) return s0;
    }
    c->z_valid = false;  // Zbar overwrites Z
    s0 = timed(ms_zb, [&]() -> ssm_status {
      hipError_t err = ssm::launch_zbar(!f64, n, nv, nb, c->w, c->z, kwb + p0 * nn, kzb + p0 * nn, st);
      return err == hipSuccess ? SSM_OK : hip_fail(err, "Zbar kernel");
    });
    if (s0 != SSM_OK) return s0;

    // Ybar_k = sum over the batch's points of mu_k(t_i) Zbar_i for k in [a_lo, k_hi]
    auto ybar_range = [&](int a_lo, int len) -> ssm_status {
      hipError_t err;
      if (p.precision == SSM_FP64)
        err = ssm::launch_sweep_f64(e, nb, len, (const double*)(ws + L.ct64) + (int64_t)p0 * L.ldct + a_lo, L.ldct,
                                    L.ldct - a_lo, (const double*)c->z, (double*)ybar, 0, st);
      else if (p.precision == SSM_FP32)
        err = ssm::launch_sweep_f32(e, nb, len, (const float*)(ws + L.ct32) + (int64_t)p0 * L.ldct + a_lo, L.ldct,
                                    L.ldct - a_lo, (const float*)c->z, (float*)ybar, 0, st);
      else if (p.precision == SSM_FP32_BF16SWEEP)
        err = ssm::launch_sweep_bf16(e, nb, len, (const float*)(ws + L.ct32) + (int64_t)p0 * L.ldct + a_lo, L.ldct,
                                     L.ldct - a_lo, (const float*)c->z, (float*)ybar, 0, st);
      else
        err = ssm::launch_sweep_bf16x3(e, nb, len, (const __bf16*)(ws + L.chit) + (int64_t)a_lo * L.ldkt + p0,
                                       (const __bf16*)(ws + L.clot) + (int64_t)a_lo * L.ldkt + p0, L.ldkt, m1 - a_lo,
                                       (int64_t)(m1 - a_lo) * L.ldkt - p0, (const float*)c->z, (float*)ybar, 0, nb,
                                       c->k3 - a_lo, st);
      return err == hipSuccess ? SSM_OK : hip_fail(err, "transposed sweep");
    };

    const int S = pl.ckpt ? pl.ckpt : m1;
    const int nseg1 = pl.ckpt ? m / S + 1 : 1;
    for (int j = nseg1 - 1; j >= 0; --j) {
      const int k_lo = j * S;
      const int k_hi = std::min(m, k_lo + S - 1);
      const char* pair1 = pl.ckpt ? c->ckpt + (size_t)(2 * j) * bb : nullptr;  // (Y_{k_lo - 1}, Y_{k_lo}) or (Y_0, Y_1)
      const int nsub = (k_hi - k_lo + L.sub) / L.sub;
      if (L.levels == 2 && nsub > 1) {
        // replay the segment from its level-1 pair, keeping (Y_{b0}, Y_{b0+1}) of every
        // sub-segment q >= 1 (b0 = k_lo + q sub - 1) in the level-2 slots; the other
        // blocks rotate through three ring slots
        const int f = ckpt_first(j, S);
        const int b_last = k_lo + (nsub - 1) * L.sub;  // Y_{b0+1} of the last sub-segment
        auto where = [&](int b) -> char* {
          if (b == f) return (char*)pair1;
          if (b == f + 1) return (char*)pair1 + bb;
          const int q = (b - k_lo + 1) / L.sub, r = (b - k_lo + 1) % L.sub;
          if (q >= 1 && q < nsub && r <= 1) return pairs2 + (size_t)(2 * q + r) * bb;
          return ring + (size_t)(b % 3) * bb;
        };
        s0 = timed(ms_rc, [&]() -> ssm_status {
          for (int b = f + 2; b <= b_last; ++b) {
            hipError_t err = cheb(where(b - 1), where(b - 2), where(b));
            if (err != hipSuccess) return hip_fail(err, "replay of T_k(A~)W for the level-2 pairs");
            ++recomputed;
          }
          return SSM_OK;
        });
        if (s0 != SSM_OK) return s0;
      }
      for (int q = nsub - 1; q >= 0; --q) {
        const int k2_lo = k_lo + q * L.sub;
        const int k2_hi = std::min(k_hi, k2_lo + L.sub - 1);
        const int b0 = k2_lo == 0 ? 0 : k2_lo - 1;
        const char* pair = q == 0 ? pair1 : pairs2 + (size_t)(2 * q) * bb;
        // block b = k - 1 of this sub-segment
        auto y_of = [&](int b) -> const char* {
          if (!pl.ckpt) return ring + (size_t)b * bb;
          if (b == b0) return pair;
          if (b == b0 + 1) return pair + bb;
          return ring + (size_t)(b - b0 - 2) * bb;
        };
        if (pl.ckpt) {
          s0 = timed(ms_rc, [&]() -> ssm_status {
            for (int b = b0 + 2; b <= k2_hi - 1; ++b) {
              hipError_t err = cheb(y_of(b - 1), y_of(b - 2), (void*)y_of(b));
              if (err != hipSuccess) return hip_fail(err, "recomputation of T_k(A~)W");
              ++recomputed;
            }
            return SSM_OK;
          });
          if (s0 != SSM_OK) return s0;
        }
        const int a_lo = k2_lo & ~3;
        s0 = timed(ms_ybar, [&]() { return ybar_range(a_lo, k2_hi - a_lo + 1); });
        if (s0 != SSM_OK) return s0;
        s0 = timed(ms_rev, [&]() -> ssm_status {
          for (int k = k2_hi; k >= std::max(k2_lo, 1); --k) {
            const char* ybk = ybar + (size_t)(k - a_lo) * bb;
            const void* x = k < m ? (const void*)lam_slot(k + 1) : nullptr;
            const void* xp = k + 2 <= m ? (const void*)lam_slot(k + 2) : nullptr;
            const char* yk1 = y_of(k - 1);
            const double coef = (k == 1 ? 1.0 : 2.0) * alpha;
            hipError_t err;
            if (f64)
              err = ssm::launch_reverse_step_f64(n, nv, c->a.row_ptr, c->a.col_idx, (const double*)c->a.values,
                                                 2 * alpha, 2 * beta, -1.0, (const double*)x, (const double*)xp,
                                                 (const double*)ybk, (double*)lam_slot(k), (const double*)yk1, coef,
                                                 grad_dev, st, c->order);
            else
              err = ssm::launch_reverse_step_f32(n, nv, c->a.row_ptr, c->a.col_idx, (const float*)c->a.values,
                                                 (float)(2 * alpha), (float)(2 * beta), -1.0f, (const float*)x,
                                                 (const float*)xp, (const float*)ybk, (float*)lam_slot(k),
                                                 (const float*)yk1, coef, grad_dev, st, c->order);
            if (err != hipSuccess) return hip_fail(err, "reverse recurrence step");
          }
          return SSM_OK;
        });
        if (s0 != SSM_OK) return s0;
        ++subsegs;
      }
    }
  }
  SSM_HIP(hipStreamSynchronize(st), "ssm_backward sync");
  c->bstats.ms_geneig = ms_ge;
  c->bstats.ms_zbar = ms_zb;
  c->bstats.ms_ybar = ms_ybar;
  c->bstats.ms_recompute = ms_rc;
  c->bstats.ms_reverse = ms_rev;
  c->bstats.ms_forward = ms_fwd;
  c->bstats.ms_total = ms_ge + ms_zb + ms_ybar + ms_rc + ms_rev + ms_fwd;
  c->bstats.segments = subsegs;
  c->bstats.recomputed = recomputed;
  c->bstats.passes = pl.passes;
  c->bstats.levels = L.levels;
  return SSM_OK;
}

ssm_status ssm_trace(ssm_ctx* c, const double* w_host, double* tr) {
  if (!c || !w_host || !tr) return fail(SSM_ERR_ARG, "ctx, w and tr must be non-NULL");
  if (!c->have_dos) return fail(SSM_ERR_STATE, "ssm_trace before ssm_dos");
  double acc = 0.0;
  for (int i = 0; i < c->p.nt; ++i) acc += w_host[i] * c->dos_host[i];
  *tr = acc;
  return SSM_OK;
}

ssm_status ssm_dgc(ssm_ctx* c, double* dgc_host, double* zeta_host) {
  if (!c || !dgc_host) return fail(SSM_ERR_ARG, "ctx and dgc must be non-NULL");
  if (!c->pl.dgc_group) return fail(SSM_ERR_STATE, "the context was made without dgc");
  if (!c->have_dgc) return fail(SSM_ERR_STATE, "ssm_dgc before ssm_dos");
  const int nt = c->p.nt, m1 = c->p.degree + 1;
  SSM_HIP(hipMemcpyAsync(dgc_host, c->dgc, sizeof(double) * nt, hipMemcpyDeviceToHost, c->stream), "copy DGC");
  if (zeta_host)
    SSM_HIP(hipMemcpyAsync(zeta_host, c->dgc + nt, sizeof(double) * m1, hipMemcpyDeviceToHost, c->stream),
            "copy moments");
  SSM_HIP(hipStreamSynchronize(c->stream), "ssm_dgc sync");
  for (int i = 0; i < nt; ++i)
    if (!std::isfinite(dgc_host[i])) return fail(SSM_ERR_NONFINITE, "DGC estimate at point %d is not finite", i);
  return SSM_OK;
}

ssm_status ssm_get_stats(const ssm_ctx* c, ssm_stats* out) {
  if (!c || !out) return fail(SSM_ERR_ARG, "ctx and out must be non-NULL");
  *out = c->stats;
  return SSM_OK;
}

ssm_status ssm_get_views(const ssm_ctx* c, ssm_views* out) {
  if (!c || !out) return fail(SSM_ERR_ARG, "ctx and out must be non-NULL");
  out->w = c->w;
  out->y = c->y;
  out->z = c->z;
  out->k_w = c->kw;
  out->k_z = c->kz;
  out->coeff = c->c64;
  out->chunk = c->pl.chunk;
  out->batch = c->pl.batch;
  out->first_point_of_last_batch = c->last_batch_start;
  out->elem_bytes = (int32_t)elem_bytes(c->p.precision);
  out->moments = c->xm;
  out->coeff_sq = c->nu;
  out->s_floor = c->pl.ress ? nullptr : c->sfloor;
  if (c->pl.ress) out->chunk = c->pl.chunk + 1;
  return SSM_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 8 weights (host).  h is sampled on the nt midpoints of the rescaled
// [-1, 1] (period 2).  Forward transform C_k - i S_k = sum_j h_j e^{-2 pi i k j/nt},
// division by G^_k = exp(-(pi k sigma^)^2 / 2) (unit-mass Gaussian) for
// |k| <= k_c, and the inverse transform back to the grid; both transforms are
// direct sums (O(nt k_c)) with the angle index reduced exactly modulo nt.  The
// division happens in the wavenumber domain so that rounding of h is amplified
// only at the wavenumbers where the Gaussian-damped DOS is itself negligible.
// ---------------------------------------------------------------------------
ssm_status ssm_trace_weights_exp(double lo, double hi, int32_t nt, int64_t n, double sigma, double beta,
                                 double spec_lo, double* w_host) {
  if (!w_host) return fail(SSM_ERR_ARG, "w must be non-NULL");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) return fail(SSM_ERR_ARG, "need finite lo < hi");
  if (nt < 1) return fail(SSM_ERR_ARG, "nt must be >= 1");
  if (n < 1) return fail(SSM_ERR_ARG, "n must be >= 1");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(SSM_ERR_ARG, "sigma must be > 0");
  if (!std::isfinite(beta)) return fail(SSM_ERR_ARG, "beta must be finite");
  if (std::isnan(spec_lo)) return fail(SSM_ERR_ARG, "spec_lo must not be NaN");
  const double dt = (hi - lo) / nt;
  const double scale = (double)n * dt * std::exp(-0.5 * (beta * sigma) * (beta * sigma));
  const double t_cut = spec_lo - beta * sigma * sigma - 10.0 * sigma;
  for (int i = 0; i < nt; ++i) {
    const double t = lo + dt * (i + 0.5);
    w_host[i] = t >= t_cut ? scale * std::exp(-beta * t) : 0.0;
    if (!std::isfinite(w_host[i])) return fail(SSM_ERR_NONFINITE, "weight %d overflows", i);
  }
  return SSM_OK;
}

ssm_status ssm_trace_weights(double lo, double hi, int32_t nt, int64_t n, double sigma, double a, double sigma_tilde,
                             ssm_scalar_fn f, void* user, double* w_host) {
  if (!f || !w_host) return fail(SSM_ERR_ARG, "f and w must be non-NULL");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) return fail(SSM_ERR_ARG, "need finite lo < hi");
  if (nt < 2) return fail(SSM_ERR_ARG, "nt must be >= 2");
  if (n < 1) return fail(SSM_ERR_ARG, "n must be >= 1");
  if (!(sigma > 0) || !std::isfinite(sigma)) return fail(SSM_ERR_ARG, "sigma must be > 0");
  if (!(a > 0 && a < 1)) return fail(SSM_ERR_ARG, "a must be in (0, 1)");
  if (!(sigma_tilde > 0) || !std::isfinite(sigma_tilde)) return fail(SSM_ERR_ARG, "sigma_tilde must be > 0");
  const double c0 = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
  const double sh = sigma / hw;
  const double cst = 0.5 * (f(c0 - hw * a, user) + f(c0 + hw * a, user));
  if (!std::isfinite(cst)) return fail(SSM_ERR_NONFINITE, "f(x(+-a)) is not finite");
  std::vector<double> h(nt);
  for (int i = 0; i < nt; ++i) {
    const double th = -1.0 + (2.0 * i + 1.0) / nt;
    const double pi_t = 0.5 * (std::erf((1.0 + a - 2.0 * th) / sigma_tilde) - std::erf((-1.0 - a - 2.0 * th) / sigma_tilde));
    if (pi_t > 1e-300) {
      const double fv = f(c0 + hw * th, user);
      h[i] = fv * pi_t + cst * (1.0 - pi_t);
    } else {
      h[i] = cst;
    }
    if (!std::isfinite(h[i])) return fail(SSM_ERR_NONFINITE, "h(t_%d) is not finite", i);
  }
  const double eta = 1e-10;
  const double kc_real = std::floor(std::sqrt(2.0 * std::log(1.0 / eta)) / (M_PI * sh));
  const int kmax = (int)std::min<double>(nt / 2, kc_real);  // k in [0, kmax]; -k handled by symmetry
  std::vector<double> cosv(nt), sinv(nt);
  for (int m = 0; m < nt; ++m) {
    cosv[m] = std::cos(2.0 * M_PI * (double)m / nt);
    sinv[m] = std::sin(2.0 * M_PI * (double)m / nt);
  }
  // coefficients of the inverse transform: f~_i = (1/nt) sum_k (P_k cos + Q_k sin)(2 pi k i / nt)
  std::vector<double> pk(kmax + 1), qk(kmax + 1);
  for (int k = 0; k <= kmax; ++k) {
    double ck = 0.0, sk = 0.0;
    long long idx = 0;
    for (int j = 0; j < nt; ++j) {
      ck += h[j] * cosv[idx];
      sk += h[j] * sinv[idx];
      idx += k;
      if (idx >= nt) idx -= nt;
    }
    const double gk = std::exp(-0.5 * (M_PI * k * sh) * (M_PI * k * sh));
    // +k and -k together; k = 0 and the Nyquist wavenumber k = nt/2 appear once
    const double mult = (k == 0 || 2 * k == nt) ? 1.0 : 2.0;
    pk[k] = mult * ck / gk;
    qk[k] = mult * sk / gk;
  }
  const double scale = (double)n * (hi - lo) / nt;  // N * dt_A
  for (int i = 0; i < nt; ++i) {
    double acc = 0.0;
    long long idx = 0;
    for (int k = 0; k <= kmax; ++k) {
      acc += pk[k] * cosv[idx] + qk[k] * sinv[idx];
      idx += i;
      if (idx >= nt) idx %= nt;
    }
    w_host[i] = scale * acc / nt;
  }
  return SSM_OK;
}

// ---------------------------------------------------------------------------
// Stage calls
// ---------------------------------------------------------------------------
ssm_status ssm_coefficients(double lo, double hi, double sigma, int64_t n, const double* t_dev, int32_t nt,
                            int32_t degree, double* c_dev, float* c32_dev, void* stream) {
  if (!t_dev || !c_dev) return fail(SSM_ERR_ARG, "t and c must be non-NULL");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) return fail(SSM_ERR_ARG, "need finite lo < hi");
  if (!(sigma > 0) || n < 1 || nt < 1 || degree < 1) return fail(SSM_ERR_ARG, "need sigma > 0, n, nt, degree >= 1");
  if (degree > kMaxDegree) return fail(SSM_ERR_UNSUPPORTED, "degree > %d", kMaxDegree);
  const double inv_norm = 1.0 / ((double)n * std::sqrt(2.0 * M_PI) * sigma);
  hipError_t e = ssm::launch_coefficients(0.5 * (lo + hi), 0.5 * (hi - lo), sigma, inv_norm, t_dev, nt, degree,
                                          n_theta_for(degree), c_dev, c32_dev, nt, (hipStream_t)stream);
  return e == hipSuccess ? SSM_OK : hip_fail(e, "coefficient kernel");
}

ssm_status ssm_gaussian_block(uint64_t seed, int64_t n, int32_t nv, int32_t dtype, void* w_dev, void* stream) {
  if (!w_dev || n < 1 || nv < 1 || (dtype != 0 && dtype != 1)) return fail(SSM_ERR_ARG, "bad arguments");
  hipError_t e = ssm::launch_gaussian_block(seed, n, nv, dtype, w_dev, (hipStream_t)stream);
  return e == hipSuccess ? SSM_OK : hip_fail(e, "W generator");
}

ssm_status ssm_chebyshev(const ssm_csr* a, double lo, double hi, int32_t precision, int32_t nv, int32_t degree,
                         const void* w, void* y, void* stream) {
  ssm_status s = check_csr(a);
  if (s != SSM_OK) return s;
  if (!w || !y) return fail(SSM_ERR_ARG, "w and y must be non-NULL");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(lo < hi)) return fail(SSM_ERR_ARG, "need finite lo < hi");
  if (nv < 4 || nv % 4 != 0) return fail(SSM_ERR_ARG, "nv must be a positive multiple of 4");
  if (degree < 0) return fail(SSM_ERR_ARG, "degree must be >= 0");
  if (precision < SSM_FP64 || precision > SSM_FP32_BF16X3) return fail(SSM_ERR_ARG, "bad precision");
  const bool f64 = precision == SSM_FP64;
  const size_t es = f64 ? 8 : 4;
  const int64_t e = a->n * nv;
  hipStream_t st = (hipStream_t)stream;
  const double alpha = 2.0 / (hi - lo), beta = -(hi + lo) / (hi - lo);
  SSM_HIP(hipMemcpyAsync(y, w, e * es, hipMemcpyDeviceToDevice, st), "copy W");
  for (int k = 1; k <= degree; ++k) {
    char* out = (char*)y + (size_t)k * e * es;
    const char* x = (char*)y + (size_t)(k - 1) * e * es;
    const char* xp = k >= 2 ? (char*)y + (size_t)(k - 2) * e * es : nullptr;
    const double aa = k == 1 ? alpha : 2 * alpha, bb = k == 1 ? beta : 2 * beta, cc = k == 1 ? 0.0 : -1.0;
    hipError_t err = f64 ? ssm::launch_cheb_step_f64(a->n, nv, a->row_ptr, a->col_idx, (const double*)a->values, aa, bb,
                                                     cc, (const double*)x, (const double*)xp, nullptr, (double*)out, st)
                         : ssm::launch_cheb_step_f32(a->n, nv, a->row_ptr, a->col_idx, (const float*)a->values,
                                                     (float)aa, (float)bb, (float)cc, (const float*)x,
                                                     (const float*)xp, nullptr, (float*)out, st);
    if (err != hipSuccess) return hip_fail(err, "Chebyshev step");
  }
  return SSM_OK;
}

ssm_status ssm_sweep(int32_t precision, int64_t e, int32_t kc, int32_t ntb, const void* c, int64_t ldc,
                     const void* y, void* z, int32_t accumulate, void* stream) {
  if (!c || !y || !z) return fail(SSM_ERR_ARG, "c, y, z must be non-NULL");
  if (e < 1 || kc < 1 || ntb < 1 || ldc < ntb) return fail(SSM_ERR_ARG, "need e, kc, ntb >= 1 and ldc >= ntb");
  const int vec = precision == SSM_FP64 ? 2 : 4;
  if (ldc % vec || e % vec) return fail(SSM_ERR_ARG, "ldc and e must be multiples of %d", vec);
  hipError_t err;
  hipStream_t st = (hipStream_t)stream;
  if (precision == SSM_FP64)
    err = ssm::launch_sweep_f64(e, kc, ntb, (const double*)c, ldc, ldc, (const double*)y, (double*)z, accumulate, st);
  else if (precision == SSM_FP32)
    err = ssm::launch_sweep_f32(e, kc, ntb, (const float*)c, ldc, ldc, (const float*)y, (float*)z, accumulate, st);
  else if (precision == SSM_FP32_BF16SWEEP)
    err = ssm::launch_sweep_bf16(e, kc, ntb, (const float*)c, ldc, ldc, (const float*)y, (float*)z, accumulate, st);
  else if (precision == SSM_FP32_BF16X3)
    return fail(SSM_ERR_ARG, "SSM_FP32_BF16X3 takes split tables: use ssm_split_coefficients and ssm_sweep_split");
  else
    return fail(SSM_ERR_ARG, "bad precision");
  return err == hipSuccess ? SSM_OK : hip_fail(err, "sweep GEMM");
}

ssm_status ssm_split_coefficients(const double* c, int64_t ldc, int32_t nt, int32_t m1, void* chi, void* clo,
                                  int64_t ldk, void* stream) {
  if (!c || !chi || !clo) return fail(SSM_ERR_ARG, "c, chi, clo must be non-NULL");
  if (nt < 1 || m1 < 1 || ldc < nt || ldk < m1 || ldk % 8) return fail(SSM_ERR_ARG, "need ldc >= nt, ldk >= m1, ldk % 8 == 0");
  if (((uintptr_t)chi | (uintptr_t)clo) % 16) return fail(SSM_ERR_ARG, "chi, clo must be 16-byte aligned");
  hipError_t err = ssm::launch_split_coefficients(c, ldc, nt, m1, (__bf16*)chi, (__bf16*)clo, ldk, nt, (hipStream_t)stream);
  return err == hipSuccess ? SSM_OK : hip_fail(err, "coefficient split kernel");
}

ssm_status ssm_sweep_split(int64_t e, int32_t kc, int32_t ntb, const void* chi, const void* clo, int64_t ldk,
                           const void* y, void* z, int32_t accumulate, int32_t k3, void* stream) {
  if (!chi || !clo || !y || !z) return fail(SSM_ERR_ARG, "chi, clo, y, z must be non-NULL");
  if (e < 1 || kc < 1 || ntb < 1 || ldk < kc || ldk % 8 || e % 4) return fail(SSM_ERR_ARG, "need e % 4 == 0, ldk >= kc, ldk % 8 == 0");
  if (((uintptr_t)chi | (uintptr_t)clo | (uintptr_t)y | (uintptr_t)z) % 16) return fail(SSM_ERR_ARG, "pointers must be 16-byte aligned");
  if ((int64_t)ntb * ldk >= ((int64_t)1 << 30)) return fail(SSM_ERR_ARG, "split tables above 2^30 entries");
  hipError_t err = ssm::launch_sweep_bf16x3(e, kc, ntb, (const __bf16*)chi, (const __bf16*)clo, ldk, ntb,
                                            (int64_t)(ntb - 1) * ldk + (kc + 7) / 8 * 8,
                                            (const float*)y, (float*)z, accumulate, k3, ntb, (hipStream_t)stream);
  return err == hipSuccess ? SSM_OK : hip_fail(err, "split sweep GEMM");
}

static ssm_status check_gram(int32_t precision, int64_t n, int32_t nv, int32_t ntb, const void* w, const void* z,
                             double* k_w, double* k_z, int32_t nseg) {
  if (!w || !z || !k_w || !k_z) return fail(SSM_ERR_ARG, "pointers must be non-NULL");
  if (n < 1 || ntb < 1 || nseg < 1) return fail(SSM_ERR_ARG, "need n, ntb, nseg >= 1");
  if (nv < 4 || nv % 4) return fail(SSM_ERR_ARG, "nv must be a positive multiple of 4");
  if (nv > kMaxNv) return fail(SSM_ERR_UNSUPPORTED, "nv > %d", kMaxNv);
  if (precision < SSM_FP64 || precision > SSM_FP32_BF16X3) return fail(SSM_ERR_ARG, "bad precision");
  return SSM_OK;
}

ssm_status ssm_gram(int32_t precision, int64_t n, int32_t nv, int32_t ntb, const void* w, const void* z, double* k_w,
                    double* k_z, int32_t nseg, double* work, void* stream) {
  ssm_status s = check_gram(precision, n, nv, ntb, w, z, k_w, k_z, nseg);
  if (s != SSM_OK) return s;
  if (!work) return fail(SSM_ERR_ARG, "pointers must be non-NULL");
  hipError_t err = ssm::launch_gram(precision != SSM_FP64, n, nv, ntb, w, z, k_w, k_z, nseg, work, (hipStream_t)stream);
  return err == hipSuccess ? SSM_OK : hip_fail(err, "Gram kernel");
}

ssm_status ssm_gram_noalloc(int32_t precision, int64_t n, int32_t nv, int32_t ntb, const void* w, const void* z,
                            double* k_w, double* k_z, int32_t nseg, void* stream) {
  ssm_status s = check_gram(precision, n, nv, ntb, w, z, k_w, k_z, nseg);
  if (s != SSM_OK) return s;
  const double need = (double)ssm::gram_scratch_slots(nseg) * ntb * 2.0 * nv * nv * sizeof(double);
  if (need > (double)SSM_NOALLOC_SCRATCH_BYTES)
    return fail(SSM_ERR_UNSUPPORTED, "ssm_gram_noalloc: %.0f bytes of partial sums exceed the %d-byte scratch array "
                "(use fewer points or segments per call)", need, SSM_NOALLOC_SCRATCH_BYTES);
  double* ptr = nullptr;
  if ((s = noalloc_scratch(&ptr)) != SSM_OK) return s;
  hipError_t err = ssm::launch_gram(precision != SSM_FP64, n, nv, ntb, w, z, k_w, k_z, nseg, ptr, (hipStream_t)stream);
  return err == hipSuccess ? SSM_OK : hip_fail(err, "Gram kernel");
}

ssm_status ssm_geneig_trace(int32_t nv, int32_t ntb, const double* k_w, const double* k_z, double g_max, double tau,
                            double rho, double* dos_dev, int32_t* ranks_dev, double* work, void* stream) {
  if (!k_w || !k_z || !dos_dev || !work) return fail(SSM_ERR_ARG, "pointers must be non-NULL");
  if (nv < 1 || ntb < 1) return fail(SSM_ERR_ARG, "need nv, ntb >= 1");
  if (nv > kMaxNv) return fail(SSM_ERR_UNSUPPORTED, "nv > %d", kMaxNv);
  if (!(g_max > 0) || !std::isfinite(tau) || !std::isfinite(rho)) return fail(SSM_ERR_ARG, "bad g_max/tau/rho");
  hipError_t err = ssm::launch_geneig_trace(nv, ntb, k_w, k_z, g_max, tau, rho, dos_dev, ranks_dev, work,
                                            (hipStream_t)stream);
  return err == hipSuccess ? SSM_OK : hip_fail(err, "Algorithm 4 kernel");
}

int64_t ssm_geneig_trace_scratch_doubles(int32_t nv, int32_t ntb) {
  if (nv < 1 || nv > kMaxNv || ntb < 1) return -1;
  return ssm::geneig_trace_scratch_doubles(nv, ntb);
}

}  // extern "C"
