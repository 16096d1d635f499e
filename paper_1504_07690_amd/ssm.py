"""Python binding of libssm: torch supplies device memory and the stream, every
step runs in the library's HIP kernels.  Names follow include/ssm.h.

Nothing here computes any part of the method: the functions check shapes,
place arrays on the device and forward pointers to the C ABI.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi as A

PRECISION = {"fp64": A.SSM_FP64, "fp32": A.SSM_FP32, "bf16": A.SSM_FP32_BF16SWEEP, "bf16x3": A.SSM_FP32_BF16X3}


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("device tensor expected")


class DeviceCSR:
    """A CSR matrix (workloads.CSR or arrays) uploaded to the device."""

    def __init__(self, n, row_ptr, col_idx, values, dtype=torch.float32, device="cuda:0"):
        self.n = int(n)
        self.row_ptr = torch.as_tensor(np.asarray(row_ptr, dtype=np.int32)).to(device)
        self.col_idx = torch.as_tensor(np.asarray(col_idx, dtype=np.int32)).to(device)
        self.values = torch.as_tensor(np.asarray(values, dtype=np.float64)).to(device=device, dtype=dtype)
        self.nnz = int(self.col_idx.numel())

    @classmethod
    def from_csr(cls, csr, dtype=torch.float32, device="cuda:0"):
        return cls(csr.n, csr.row_ptr, csr.col_idx, csr.values, dtype, device)

    def struct(self) -> A.ssm_csr:
        return A.ssm_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                         self.values.data_ptr())


METHOD = {"ss": 0, "ress": 1}


def _params(lo, hi, sigma, nv, degree, nt, precision, tau, rho, seed, ckpt_every=0, dgc=False, method="ss",
            nv_hybrid=0, floor_scale=0.0, plan=None, lattice=None) -> A.ssm_params:
    batch, chunk = plan if plan is not None else (0, 0)
    lat = (C.c_int32 * 3)(*(lattice if lattice is not None else (0, 0, 0)))
    return A.ssm_params(float(lo), float(hi), float(sigma), float(tau), float(rho), int(nv), int(degree),
                        int(nt), int(PRECISION[precision]), int(seed) & 0xFFFFFFFFFFFFFFFF, int(ckpt_every),
                        int(bool(dgc)), int(METHOD[method]), int(nv_hybrid), float(floor_scale), int(batch),
                        int(chunk), lat)


def workspace_size(csr: DeviceCSR, *, lo, hi, sigma, nv, degree, nt, precision="fp32", tau=1e-7, rho=1e-3,
                   seed=0, budget=0, ckpt_every=0, dgc=False, method="ss", nv_hybrid=0, floor_scale=0.0,
                   plan=None, lattice=None) -> int:
    out = C.c_size_t(0)
    p = _params(lo, hi, sigma, nv, degree, nt, precision, tau, rho, seed, ckpt_every, dgc, method, nv_hybrid,
                floor_scale, plan, lattice)
    A.check(A.lib.ssm_workspace_size(C.byref(csr.struct()), C.byref(p), C.c_size_t(budget), C.byref(out)),
            "ssm_workspace_size")
    return int(out.value)


class SSM:
    """One context of the spectrum sweeping method on the device: Algorithm 5 (method "ss")
    or Algorithm 7 (method "ress", with nv_hybrid columns of W~ for the correction of
    Algorithm 6; w then has nv + nv_hybrid columns)."""

    def __init__(self, csr: DeviceCSR, *, lo, hi, sigma, nv, degree, t, precision="fp32", tau=1e-7, rho=1e-3,
                 seed=0, w: torch.Tensor | None = None, budget=0, ckpt_every=0, dgc=False, method="ss",
                 nv_hybrid=0, floor_scale=0.0, plan=None, lattice=None, device="cuda:0"):
        self.csr = csr
        self.t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
        self.nt = int(self.t.size)
        self.nv = int(nv)
        self.precision = precision
        self.elem = torch.float64 if precision == "fp64" else torch.float32
        if w is not None:
            _require_cuda(w)
            cols = nv + nv_hybrid
            if w.dtype != self.elem or tuple(w.shape) != (csr.n, cols) or not w.is_contiguous():
                raise ValueError(f"w must be a contiguous {self.elem} tensor of shape ({csr.n}, {cols})")
        self.w_in = w
        self.degree = int(degree)
        self.method = method
        self.nv_hybrid = int(nv_hybrid)
        self.params = _params(lo, hi, sigma, nv, degree, self.nt, precision, tau, rho, seed, ckpt_every, dgc,
                              method, nv_hybrid, floor_scale, plan, lattice)
        size = C.c_size_t(0)
        A.check(A.lib.ssm_workspace_size(C.byref(csr.struct()), C.byref(self.params), C.c_size_t(budget),
                                         C.byref(size)), "ssm_workspace_size")
        if budget:
            size = C.c_size_t(budget)
        self.ws = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=device)
        self._size = int(size.value)
        self._off = (-self.ws.data_ptr()) % 256
        self._ctx = C.c_void_p(0)
        self._create()

    def _create(self):
        tp = self.t.ctypes.data_as(C.POINTER(C.c_double))
        A.check(A.lib.ssm_create(C.byref(self.csr.struct()), C.byref(self.params), tp, _ptr(self.w_in),
                                 C.c_void_p(self.ws.data_ptr() + self._off), C.c_size_t(self._size), _stream(),
                                 C.byref(self._ctx)), "ssm_create")

    def reset(self):
        """Destroy the context and create it again on the same workspace: the set-up of
        ssm_create (the coefficients of Algorithm 1, W, the split tables) runs again."""
        self.close()
        self._create()

    def dos(self):
        """(dos, r1, r2): the DOS estimate at the sweep points (A's units) and kept counts."""
        out = np.zeros(self.nt, dtype=np.float64)
        ranks = np.zeros(2 * self.nt, dtype=np.int32)
        A.check(A.lib.ssm_dos(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double)),
                              ranks.ctypes.data_as(C.POINTER(C.c_int32))), "ssm_dos")
        return out, ranks[: self.nt].copy(), ranks[self.nt:].copy()

    def dgc(self):
        """(dgc, zeta): the DGC estimate of Algorithm 2 at the sweep points and the moments
        zeta_0..zeta_M, from the last dos() (context made with dgc=True)."""
        out = np.zeros(self.nt, dtype=np.float64)
        zeta = np.zeros(self.degree + 1, dtype=np.float64)
        A.check(A.lib.ssm_dgc(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double)),
                              zeta.ctypes.data_as(C.POINTER(C.c_double))), "ssm_dgc")
        return out, zeta

    def trace(self, w) -> float:
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        tr = C.c_double(0.0)
        A.check(A.lib.ssm_trace(self._ctx, w.ctypes.data_as(C.POINTER(C.c_double)), C.byref(tr)), "ssm_trace")
        return tr.value

    def stats(self) -> dict:
        s = A.ssm_stats()
        A.check(A.lib.ssm_get_stats(self._ctx, C.byref(s)), "ssm_get_stats")
        return {k: getattr(s, k) for k, _ in A.ssm_stats._fields_}

    def _view(self, ptr, count, dtype):
        off = ptr - self.ws.data_ptr()
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.ws[off: off + nbytes].view(dtype)

    def views(self) -> dict:
        """Device views into the context's buffers (see ssm_get_views)."""
        v = A.ssm_views()
        A.check(A.lib.ssm_get_views(self._ctx, C.byref(v)), "ssm_get_views")
        n, nv, nt = self.csr.n, self.nv, self.nt
        nvp = nv + self.nv_hybrid  # columns of the block the recurrence runs on
        e = n * nvp
        m1 = self.params.degree + 1
        ldc = (nt + 3) // 4 * 4
        out = {
            "y": self._view(v.y, v.chunk * e, self.elem).view(v.chunk, n, nvp),
            "k_w": self._view(v.k_w, nt * nv * nv, torch.float64).view(nt, nv, nv),
            "k_z": self._view(v.k_z, nt * nv * nv, torch.float64).view(nt, nv, nv),
            "coeff": self._view(v.coeff, m1 * ldc, torch.float64).view(m1, ldc)[:, :nt],
            "chunk": v.chunk, "batch": v.batch, "first_point_of_last_batch": v.first_point_of_last_batch,
        }
        if v.z:
            out["z"] = self._view(v.z, v.batch * e, self.elem).view(v.batch, n, nvp)
        if v.moments:
            out["moments"] = self._view(v.moments, m1 * nvp * nvp, torch.float64).view(m1, nvp, nvp)
            out["coeff_sq"] = self._view(v.coeff_sq, m1 * ldc, torch.float64).view(m1, ldc)[:, :nt]
        if v.s_floor:
            out["s_floor"] = self._view(v.s_floor, nt, torch.float64)
        out["w"] = self.w_in if self.w_in is not None else self._view(v.w, e, self.elem).view(n, nvp)
        return out

    def backward(self, dos_bar) -> torch.Tensor:
        """Gradient of sum_i dos_bar[i] dos[i] w.r.t. the stored values (ssm_backward):
        a float64 device tensor of nnz entries.  Overwrites the context's Z blocks; a later
        backward forms them again."""
        dos_bar = np.ascontiguousarray(np.asarray(dos_bar, dtype=np.float64))
        assert dos_bar.shape == (self.nt,)
        size = C.c_size_t(0)
        A.check(A.lib.ssm_backward_workspace_size(self._ctx, C.byref(size)), "ssm_backward_workspace_size")
        ws = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=self.ws.device)
        base = ws.data_ptr() + (-ws.data_ptr()) % 256
        grad = torch.empty(self.csr.nnz, dtype=torch.float64, device=self.ws.device)
        A.check(A.lib.ssm_backward(self._ctx, dos_bar.ctypes.data_as(C.POINTER(C.c_double)), _ptr(grad),
                                   C.c_void_p(base), C.c_size_t(int(size.value))), "ssm_backward")
        return grad

    def backward_stats(self) -> dict:
        s = A.ssm_backward_stats()
        A.check(A.lib.ssm_get_backward_stats(self._ctx, C.byref(s)), "ssm_get_backward_stats")
        return {k: getattr(s, k) for k, _ in A.ssm_backward_stats._fields_}

    def close(self):
        if self._ctx:
            A.check(A.lib.ssm_destroy(self._ctx), "ssm_destroy")
            self._ctx = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SpectrumSweep(torch.autograd.Function):
    """values (nnz, device) -> DOS estimate at the sweep points (float64, device).

    backward runs the library's adjoint (ssm_backward): the gradient of
    sum_i grad_out[i] dos[i] with respect to every stored value."""

    @staticmethod
    def forward(fctx, values, row_ptr, col_idx, n, opts):
        csr = DeviceCSR.__new__(DeviceCSR)
        csr.n, csr.row_ptr, csr.col_idx = int(n), row_ptr, col_idx
        csr.values = values.detach().contiguous()
        csr.nnz = int(col_idx.numel())
        obj = SSM(csr, **opts)
        dos, _, _ = obj.dos()
        fctx.obj = obj
        fctx.vdtype = values.dtype
        return torch.as_tensor(dos, device=values.device)

    @staticmethod
    def backward(fctx, grad_out):
        grad = fctx.obj.backward(grad_out.detach().double().cpu().numpy())
        fctx.obj.close()
        return grad.to(fctx.vdtype), None, None, None, None


def dos_autograd(values: torch.Tensor, row_ptr: torch.Tensor, col_idx: torch.Tensor, n: int, **opts) -> torch.Tensor:
    """Differentiable DOS: opts are SSM's keyword arguments (lo, hi, sigma, nv, degree, t, ...)."""
    return SpectrumSweep.apply(values, row_ptr, col_idx, n, opts)


def trace_weights_exp(beta, *, lo, hi, nt, n, sigma, spec_lo=-np.inf) -> np.ndarray:
    """Weights of Tr exp(-beta A) by the exact real-line deconvolution, zero below
    spec_lo - beta sigma^2 - 10 sigma (ssm_trace_weights_exp)."""
    w = np.zeros(int(nt), dtype=np.float64)
    A.check(A.lib.ssm_trace_weights_exp(float(lo), float(hi), int(nt), int(n), float(sigma), float(beta),
                                        float(spec_lo), w.ctypes.data_as(C.POINTER(C.c_double))),
            "ssm_trace_weights_exp")
    return w


def trace_weights(f, *, lo, hi, nt, n, sigma, a=0.9, sigma_tilde=0.016) -> np.ndarray:
    """Algorithm 8 weights (host, in the library): Tr f(A) ~= sum_i w_i dos_i."""
    cb = A.SCALAR_FN(lambda x, _u: float(f(x)))
    w = np.zeros(int(nt), dtype=np.float64)
    A.check(A.lib.ssm_trace_weights(float(lo), float(hi), int(nt), int(n), float(sigma), float(a),
                                    float(sigma_tilde), cb, None, w.ctypes.data_as(C.POINTER(C.c_double))),
            "ssm_trace_weights")
    return w


# ----------------------------------------------------------------------------
# Stage calls (each enqueues on torch's current stream)
# ----------------------------------------------------------------------------
def coefficients(lo, hi, sigma, n, t: torch.Tensor, degree, out: torch.Tensor, out32: torch.Tensor | None = None):
    _require_cuda(t, out, out32)
    nt = t.numel()
    assert t.dtype == torch.float64 and out.dtype == torch.float64 and out.numel() >= (degree + 1) * nt
    A.check(A.lib.ssm_coefficients(float(lo), float(hi), float(sigma), int(n), _ptr(t), int(nt), int(degree),
                                   _ptr(out), _ptr(out32), _stream()), "ssm_coefficients")


def gaussian_block(seed, out: torch.Tensor):
    _require_cuda(out)
    n, nv = out.shape
    dtype = {torch.float64: 0, torch.float32: 1}[out.dtype]
    A.check(A.lib.ssm_gaussian_block(int(seed) & 0xFFFFFFFFFFFFFFFF, int(n), int(nv), dtype, _ptr(out), _stream()),
            "ssm_gaussian_block")


def chebyshev(csr: DeviceCSR, lo, hi, precision, w: torch.Tensor, y: torch.Tensor):
    _require_cuda(w, y)
    m1, n, nv = y.shape
    A.check(A.lib.ssm_chebyshev(C.byref(csr.struct()), float(lo), float(hi), PRECISION[precision], int(nv),
                                int(m1 - 1), _ptr(w), _ptr(y), _stream()), "ssm_chebyshev")


def sweep(precision, c: torch.Tensor, y: torch.Tensor, z: torch.Tensor, accumulate=False):
    """z[i] (+)= sum_k c[k, i] y[k] with c (kc x ldc), y (kc x ...), z (ntb x ...)."""
    _require_cuda(c, y, z)
    kc, ldc = c.shape
    ntb = z.shape[0]
    e = y[0].numel()
    A.check(A.lib.ssm_sweep(PRECISION[precision], int(e), int(kc), int(ntb), _ptr(c), int(ldc), _ptr(y), _ptr(z),
                            int(bool(accumulate)), _stream()), "ssm_sweep")


def split_coefficients(c: torch.Tensor, nt: int, ldk: int):
    """Split tables (chi, clo) of the FP64 coefficient table c (m1 x ldc) for bf16x3."""
    _require_cuda(c)
    m1, ldc = c.shape
    chi = torch.empty(nt * ldk, dtype=torch.bfloat16, device=c.device)
    clo = torch.empty_like(chi)
    A.check(A.lib.ssm_split_coefficients(_ptr(c), int(ldc), int(nt), int(m1), _ptr(chi), _ptr(clo), int(ldk),
                                         _stream()), "ssm_split_coefficients")
    return chi.view(nt, ldk), clo.view(nt, ldk)


def sweep_split(chi: torch.Tensor, clo: torch.Tensor, y: torch.Tensor, z: torch.Tensor, kc=None, accumulate=False,
                k3=None):
    """z[i] (+)= sum_{k<kc} c[k, i] y[k] in the bf16x3 arithmetic, c given by its split tables;
    degrees k >= k3 (rounded up to a multiple of 32) take the single product Chi Yhi."""
    _require_cuda(chi, clo, y, z)
    ntb_tab, ldk = chi.shape
    kc = y.shape[0] if kc is None else kc
    ntb = z.shape[0]
    assert ntb <= ntb_tab
    e = y[0].numel()
    k3 = kc if k3 is None else int(k3)
    A.check(A.lib.ssm_sweep_split(int(e), int(kc), int(ntb), _ptr(chi), _ptr(clo), int(ldk), _ptr(y), _ptr(z),
                                  int(bool(accumulate)), k3, _stream()), "ssm_sweep_split")


def gram(precision, w: torch.Tensor, z: torch.Tensor, k_w: torch.Tensor, k_z: torch.Tensor, nseg=1):
    _require_cuda(w, z, k_w, k_z)
    n, nv = w.shape
    ntb = z.shape[0]
    scratch = torch.empty(4 * nseg * ntb * 2 * nv * nv, dtype=torch.float64, device=w.device)
    A.check(A.lib.ssm_gram(PRECISION[precision], int(n), int(nv), int(ntb), _ptr(w), _ptr(z), _ptr(k_w), _ptr(k_z),
                           int(nseg), _ptr(scratch), _stream()), "ssm_gram")
    return scratch


def gram_noalloc(precision, w: torch.Tensor, z: torch.Tensor, k_w: torch.Tensor, k_z: torch.Tensor, nseg=1):
    """ssm_gram_noalloc: the Gram stage call with the library's own static scratch array."""
    _require_cuda(w, z, k_w, k_z)
    n, nv = w.shape
    ntb = z.shape[0]
    A.check(A.lib.ssm_gram_noalloc(PRECISION[precision], int(n), int(nv), int(ntb), _ptr(w), _ptr(z), _ptr(k_w),
                                   _ptr(k_z), int(nseg), _stream()), "ssm_gram_noalloc")


def geneig_trace(k_w: torch.Tensor, k_z: torch.Tensor, g_max, tau, rho, dos: torch.Tensor,
                 ranks: torch.Tensor | None = None):
    _require_cuda(k_w, k_z, dos, ranks)
    ntb, nv, _ = k_w.shape
    size = A.lib.ssm_geneig_trace_scratch_doubles(int(nv), int(ntb))
    if size < 0:
        raise ValueError(f"ssm_geneig_trace: unsupported nv={nv}, ntb={ntb}")
    scratch = torch.empty(size, dtype=torch.float64, device=k_w.device)
    A.check(A.lib.ssm_geneig_trace(int(nv), int(ntb), _ptr(k_w), _ptr(k_z), float(g_max), float(tau), float(rho),
                                   _ptr(dos), _ptr(ranks), _ptr(scratch), _stream()), "ssm_geneig_trace")
    return scratch
