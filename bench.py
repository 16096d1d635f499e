"""Benchmark of the spectrum sweeping DOS (Algorithm 5) on one MI355X.

Workload: the 3D Anderson model on a 64^3 periodic lattice (N = 262144, hopping -1,
disorder uniform in [-2, 2]), N_v = 80, Chebyshev degree M = 1000, N_t = 1000
midpoint sweep points, sigma = 0.01 in the rescaled variable.  Default path: FP32
recurrence, split-BF16 (three BF16 MFMA products, FP32 accumulation) sweep, FP64
Gram / Algorithm 4; the FP64, FP32 and plain-BF16 paths are timed beside it with
their DOS L1 against the FP64 path.  One step = the whole path: ssm_create's set-up on
the context's workspace (the coefficients of Algorithm 1, W, the split tables) and one
ssm_dos.  The adjoint (ssm_backward) of the
measured path is timed once after the steps, and so is one ssm_dos that also forms the
DGC estimate of Algorithm 2 from the same recurrence, and RESS-DGC (Algorithm 7, FP64)
with N_v = 80 and with 40 + 40 vectors (hybrid correction of Algorithm 6; also with an FP32
recurrence), the random-graph
workload's whole DOS (SS-DGC, and RESS-DGC with an FP32 recurrence), the 27-point workload's
recurrence rate and its whole DOS by RESS-DGC (FP32 recurrence), the 32 x 32 workload (device
paths against the oracle's whole run on one host thread), and the copy and GEMM rates torch's
own kernels reach on the GPU.  The oracle's baseline runs first, on the host cores.

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3|bf16|fp64]
                    [--no-fp64] [--no-bf16] [--no-cpu-baseline] [--no-adjoint] [--no-dgc] [--no-ress]
                    [--no-large]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cheb block-SpMM GB/s (% HBM peak); SSM DOS time at fixed L1 error"
HBM_PEAK_GBPS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}


def pmc_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed FETCH_SIZE / WRITE_SIZE
    record (each scaled by what the counter reads for a plain copy of known size),
    or None when there is no record or the kernel's source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_point_worker(args):
    """One sweep point of the oracle on the first `steps` blocks (a process of the pool):
    seconds for its coefficients, per block of its sweep, and for its Gram matrices and
    Algorithm 4.  One thread per process."""
    cfg, point, steps = args
    from threadpoolctl import threadpool_limits

    from oracle import ssm_oracle as O
    from paper_1504_07690_amd import workloads as WL
    with threadpool_limits(1):
        wl = WL.make_workload(cfg)
        w = wl.w()
        blocks = [v for _, v in O.chebyshev_blocks(wl.a, w, steps, wl.lo, wl.hi)]
        t0 = time.perf_counter()
        mu = O.dgc_coefficients(wl.t[[point]], wl.degree, wl.sigma, wl.a.n, wl.lo, wl.hi)
        t_coef = time.perf_counter() - t0
        t0 = time.perf_counter()
        z = O.sweep(mu[: steps + 1], iter(blocks))
        t_axpy = (time.perf_counter() - t0) / (steps + 1)
        t0 = time.perf_counter()
        kw, kz = O.gram(w, z[0])
        O.geneig_trace(kw, kz, O.range_bound(wl.sigma, wl.a.n))
        t_point = time.perf_counter() - t0
    return t_coef, t_axpy, t_point


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(cfg, sample_steps=16, max_workers=16):
    """The oracle, as it stands, on a bounded sample of the same workload, on the host's
    cores (run before anything touches the GPU: the pool forks).  The recurrence's sparse
    products are sequential (the oracle's, one core): timed on `sample_steps` steps.  The
    sweep points are independent given the blocks: one point per process of a pool of up to
    16 processes (the host's share), each timing its coefficients, its sweep over the sample
    blocks and its Gram matrices and Algorithm 4 while the others run.  Extrapolated to M
    steps and N_t points (seconds per DOS)."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_limits

    from oracle import ssm_oracle as O
    from paper_1504_07690_amd import workloads as WL
    model, nproc = host_cpu()
    workers = max(1, min(max_workers, nproc))
    wl = WL.make_workload(cfg)
    with threadpool_limits(1):
        w = wl.w()
        it = O.chebyshev_blocks(wl.a, w, sample_steps, wl.lo, wl.hi)
        next(it)
        t0 = time.perf_counter()
        for _ in it:
            pass
        t_step = (time.perf_counter() - t0) / sample_steps
    del w, it
    pts = np.linspace(0, wl.nt - 1, workers).astype(int)
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_point_worker, [(cfg, int(p), sample_steps) for p in pts])
    t_coef, t_axpy, t_point = (float(np.mean([r[k] for r in res])) for k in range(3))
    m1 = wl.degree + 1
    per_point = t_coef + t_axpy * m1 + t_point
    total = t_step * wl.degree + per_point * wl.nt / workers
    return {
        "value": total, "unit": "s", "cores": workers, "kind": "oracle",
        "sample": (f"host {model}, {nproc} cores visible, {workers} used: {sample_steps} Chebyshev steps "
                   f"(sequential sparse products, {t_step:.3g} s/step); {workers} sweep points in {workers} "
                   f"processes (one thread each), each its coefficients ({t_coef:.3g} s), its sweep over the "
                   f"{sample_steps + 1} blocks ({t_axpy:.3g} s/block), Gram + Algorithm 4 ({t_point:.3g} s); "
                   f"extrapolated to M={wl.degree} steps and N_t={wl.nt} points over {workers} processes"),
    }


def spmm_bytes_models(n, nnz, nv, es):
    """Bytes of one Chebyshev step: compulsory (Y_k and Y_{k-1} read once, Y_{k+1} written,
    the CSR read once) and gather-inclusive (Y_k read once per stored entry instead)."""
    e = n * nv
    compulsory = 3 * e * es + nnz * (4 + es) + (n + 1) * 4
    gather = compulsory - e * es + nnz * nv * es
    return compulsory, gather


def machine_rates(torch, dev):
    """What the GPU reaches on plain library work, beside the vendor peaks: a device-to-device
    copy of 4 GiB (bytes read + written per second) and square GEMMs in BF16 and FP64 (torch's
    BLAS), each the best of 5 launches."""
    def best(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts)
    src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    t_copy = best(lambda: dst.copy_(src))
    del src, dst
    out = {"copy_GBps": 2 * (4 << 30) / t_copy / 1e9}
    for name, dt, nn in (("bf16_gemm_TFLOPs", torch.bfloat16, 8192), ("fp64_gemm_TFLOPs", torch.float64, 8192)):
        a = torch.randn(nn, nn, dtype=dt, device=dev)
        b = torch.randn(nn, nn, dtype=dt, device=dev)
        t = best(lambda: torch.matmul(a, b))
        out[name] = 2 * nn ** 3 / t / 1e12
        del a, b
    torch.cuda.empty_cache()
    return out


def geneig_scaling(S, torch, dev, cases=((80, 2048), (128, 2048), (256, 2048))):
    """Algorithm 4 alone (ssm_geneig_trace), N_t = 2048 points (one launch group of the
    tridiagonal path), on seeded pencils K_W = G^T G, K_Z = 1e-4 H^T H with G, H Gaussian
    (3 N_v x N_v per point), range bound 1: ms per 1000 points, best of 3 launches."""
    out = {}
    gen = torch.Generator(device=dev)
    for nv, ntb in cases:
        gen.manual_seed(1000 + nv)
        kw = torch.empty(ntb, nv, nv, dtype=torch.float64, device=dev)
        kz = torch.empty_like(kw)
        for i0 in range(0, ntb, 256):  # in slices, to bound the temporaries
            k = min(256, ntb - i0)
            g = torch.randn(k, 3 * nv, nv, dtype=torch.float64, device=dev, generator=gen)
            kw[i0:i0 + k] = torch.bmm(g.transpose(1, 2).contiguous(), g)
            h = torch.randn(k, 3 * nv, nv, dtype=torch.float64, device=dev, generator=gen)
            kz[i0:i0 + k] = 1e-4 * torch.bmm(h.transpose(1, 2).contiguous(), h)
            del g, h
        dos = torch.empty(ntb, dtype=torch.float64, device=dev)
        ranks = torch.empty(2 * ntb, dtype=torch.int32, device=dev)
        S.geneig_trace(kw, kz, 1.0, 1e-7, 1e-3, dos, ranks)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            S.geneig_trace(kw, kz, 1.0, 1e-7, 1e-3, dos, ranks)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[f"nv{nv}"] = {"points": ntb, "ms_per_1000_points": min(ts) * 1000 / ntb,
                          "path": "tridiagonal" if nv > 48 else "jacobi",
                          "mean_r1": float(ranks[:ntb].double().mean()), "mean_r2": float(ranks[ntb:].double().mean())}
        log(f"Algorithm 4, N_v = {nv}: {out[f'nv{nv}']['ms_per_1000_points']:.1f} ms per 1000 points")
        del kw, kz
    torch.cuda.empty_cache()
    return out


def cpu_baseline_small():
    """The oracle's whole SS-DGC on the 32 x 32 random Laplacian (N = 1024, N_v = 40, M = 200,
    N_t = 200) on one host thread, the paper's setting: seconds and the estimate."""
    from threadpoolctl import threadpool_limits

    from oracle import ssm_oracle as O
    from paper_1504_07690_amd import workloads as WL
    wl = WL.make_workload(1)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = O.ss_dgc(wl.a, wl.w(), wl.t, wl.degree, wl.sigma, wl.lo, wl.hi)
        return time.perf_counter() - t0, ref["dos"]


def small_workload(S, WL, torch, dev, oracle_small):
    """The 32 x 32 random Laplacian (N = 1024, N_v = 40, M = 200, N_t = 200): the device's FP64 and
    split-BF16 paths, against the oracle's run of the baseline leg (one host thread) on the
    same W when it was taken."""
    wl = WL.make_workload(1)
    w = wl.w()
    entry = {"workload": wl.name, "n": wl.a.n, "nv": wl.nv, "degree": wl.degree, "nt": wl.nt}
    ref = None
    if oracle_small is not None:
        entry["oracle_s_one_thread"], ref = oracle_small
    for precision in ("fp64", "bf16x3"):
        dt = torch.float64 if precision == "fp64" else torch.float32
        csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=dev)
        ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t,
                    precision=precision, w=torch.tensor(w, dtype=dt, device=dev), device=dev)
        ctx.dos()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dos, _, _ = ctx.dos()
        t_dev = time.perf_counter() - t0
        ctx.close()
        entry[f"{precision}_ms_per_dos"] = t_dev * 1e3
        if ref is not None:
            entry[f"{precision}_dos_l1_vs_oracle"] = float(np.abs(dos - ref).sum() / np.abs(ref).sum())
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3", "bf16", "fp64"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the timing of the adjoint (ssm_backward)")
    ap.add_argument("--no-dgc", action="store_true", help="skip the run with the DGC moments (Algorithm 2)")
    ap.add_argument("--no-ress", action="store_true", help="skip the RESS-DGC runs (Algorithm 7)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the random-graph DOS and the 27-point recurrence rate")
    ap.add_argument("--only-geneig", action="store_true",
                    help="time Algorithm 4 alone at N_v = 80, 128, 256 and print that JSON only")
    ap.add_argument("--only-stencil27", action="store_true",
                    help="time the 27-point lattice's recurrence alone (degree 400, 8 points) and print "
                         "that JSON only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="start with a plain 1 GiB device-to-device copy (a known-size kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the sweep-point batches would shard across GPUs with no "
              "communication until a final gather, and that path is not built; use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    # the oracle's baseline first: its process pool forks before anything touches the GPU
    baseline = None
    oracle_small = None
    if not args.no_cpu_baseline and not args.only_geneig and not args.only_stencil27:
        log("timing the oracle on a bounded sample on the host cores ...")
        t0 = time.time()
        baseline = cpu_baseline(2)
        log(f"oracle baseline: {baseline['value']:.4g} s per DOS extrapolated ({time.time() - t0:.1f} s)")
        if not args.no_large:
            oracle_small = cpu_baseline_small()
            baseline["small_workload_s_one_thread"] = oracle_small[0]

    import torch

    from paper_1504_07690_amd import ssm as S
    from paper_1504_07690_amd import workloads as WL

    dev = "cuda:0"
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.only_geneig:
        print(json.dumps({"geneig": geneig_scaling(S, torch, dev)}), flush=True)
        return
    if args.only_stencil27:
        free, _ = torch.cuda.mem_get_info()
        print(json.dumps({"stencil27_recurrence": stencil27_recurrence(S, WL, torch, dev,
                                                                        int(free - 12 * (1 << 30)))}), flush=True)
        return
    t0 = time.time()
    wl = WL.make_workload(2)
    log(f"workload {wl.name}: n={wl.a.n} nnz={wl.a.nnz} nv={wl.nv} M={wl.degree} nt={wl.nt} "
        f"[{wl.lo:.4f}, {wl.hi:.4f}] ({time.time() - t0:.1f} s)")
    n, nv, m = wl.a.n, wl.nv, wl.degree
    e = n * nv

    adjoint = {}
    dgc_out = {}

    def run(precision, steps, warmup, budget=0, with_adjoint=False, dgc=False):
        """`steps` timed steps, each the whole path: ssm_create's set-up on the context's
        workspace (coefficients of Algorithm 1, W, split tables) and ssm_dos."""
        dt = torch.float64 if precision == "fp64" else torch.float32
        csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=dev)
        ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=m, t=wl.t, precision=precision,
                    seed=wl.seed, budget=budget, dgc=dgc, lattice=wl.lattice, device=dev)
        for _ in range(warmup):
            ctx.reset()
            ctx.dos()
        torch.cuda.synchronize()
        t_setup = 0.0
        t_start = time.perf_counter()
        for _ in range(steps):
            t_s = time.perf_counter()
            ctx.reset()  # ssm_create synchronises before it returns
            t_setup += time.perf_counter() - t_s
            dos, r1, r2 = ctx.dos()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t_start) * 1e3 / max(steps, 1)
        ms_setup = t_setup * 1e3 / max(steps, 1)
        st = ctx.stats()
        st["ms_setup"] = ms_setup
        if dgc:
            dgc_out["dos"], _ = ctx.dgc()
        if with_adjoint:
            # gradient of sum_i dos_bar_i dos_i w.r.t. the nnz values, dos_bar weighting the
            # resolved points (estimate above 1e-2 of its maximum): one warm-up, one timed
            dos_bar = np.random.default_rng(5).uniform(0.0, 1.0, wl.nt) * (dos > 1e-2 * dos.max())
            ctx.backward(dos_bar)
            ctx.dos()
            torch.cuda.synchronize()
            t_b = time.perf_counter()
            g = ctx.backward(dos_bar)
            torch.cuda.synchronize()
            adjoint.update(ms=(time.perf_counter() - t_b) * 1e3, phases_ms=ctx.backward_stats(),
                           grad_finite=bool(torch.isfinite(g).all().item()))
            del g
            log(f"{precision} adjoint: {adjoint['ms']:.1f} ms  phases {adjoint['phases_ms']}")
        ctx.close()
        del ctx, csr
        torch.cuda.empty_cache()
        log(f"{precision}: {ms:.1f} ms per step (set-up {ms_setup:.2f} ms + DOS)  phases {st}")
        return ms, dos, r1, r2, st

    def budget_left(reserve_gib=6):
        free, _ = torch.cuda.mem_get_info()
        return int(free - reserve_gib * (1 << 30))

    ms, dos, r1, r2, st = run(args.precision, args.steps, args.warmup, budget=0,
                              with_adjoint=not args.no_adjoint)
    es = 8 if args.precision == "fp64" else 4

    spmm_bytes, _ = spmm_bytes_models(n, wl.a.nnz, nv, es)
    spmm_us = st["ms_recurrence"] * 1e3 / st["spmm_launches"]
    spmm_gbps = spmm_bytes / (spmm_us * 1e-6) / 1e9
    # sweep GEMM: 2 e (M+1) N_t flops
    sweep_flops = 2.0 * e * (m + 1) * wl.nt
    sweep_tflops = sweep_flops / (st["ms_sweep"] * 1e-3) / 1e12
    # Gram: the symmetric K_Z and K_W need N N_v (N_v + 1) multiply-adds each per point; the
    # kernel issues the upper 16 x 16 blocks (2 N N_v (N_v + 16) flops per point)
    gram_flops = 2.0 * n * nv * (nv + 1) * wl.nt
    phases = {k: st[k] for k in ("ms_setup", "ms_total", "ms_recurrence", "ms_sweep", "ms_gram", "ms_geneig")}
    dom = max(("sweep", st["ms_sweep"]), ("spmm", st["ms_recurrence"]), ("gram", st["ms_gram"]),
              key=lambda kv: kv[1])[0]
    if dom == "sweep":
        per_launch_ms = st["ms_sweep"] / st["sweep_launches"]
        roof = {"kernel": f"sweep_{args.precision}_kernel", "bound": "mfma",
                "achieved": sweep_flops / st["sweep_launches"] / (per_launch_ms * 1e-3) / 1e12,
                "peak": MFMA_PEAK_TFLOPS[args.precision], "unit": "TFLOP/s", "traffic": None}
    elif dom == "spmm":
        roof = {"kernel": "cheb_step_kernel", "bound": "hbm", "achieved": spmm_gbps, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "traffic": None}
    else:
        roof = {"kernel": "gram_kernel", "bound": "mfma",
                "achieved": gram_flops / (st["ms_gram"] * 1e-3) / 1e12, "peak": MFMA_PEAK_TFLOPS["fp64"],
                "unit": "TFLOP/s", "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = pmc_traffic(roof["kernel"])
    if args.precision == "bf16x3" and dom == "sweep":
        # achieved counts the algorithmic flops once; the matrix cores run three BF16 products
        # on the degrees below split_k3 (rounded up to 32) and one on the rest
        k3r = min(m + 1, -(-st["split_k3"] // 32) * 32)
        roof["mfma_issue_frac"] = roof["frac"] * (3.0 * k3r + (m + 1 - k3r)) / (m + 1)

    out = {
        "metric": METRIC, "value": ms / 1e3, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16x3": "bf16x3", "bf16": "bf16", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "nnz": wl.a.nnz, "nv": nv, "degree": m, "nt": wl.nt,
                   "sigma_hat": wl.sigma_hat, "recurrence_sweep": args.precision, "gram_eig": "fp64",
                   "lattice": list(wl.lattice),
                   "step": "ssm_create set-up (coefficients, W, split tables) + ssm_dos",
                   "plan": {"passes": st["passes"], "chunk": st["chunk"], "batch": st["batch"]}},
        "spmm": {"GBps": spmm_gbps, "frac_hbm": spmm_gbps / HBM_PEAK_GBPS, "bytes_per_launch": spmm_bytes,
                 "us_per_launch": spmm_us, "launches": st["spmm_launches"]},
        "sweep": {"TFLOPs": sweep_tflops, "frac_mfma": sweep_tflops / MFMA_PEAK_TFLOPS[args.precision],
                  "three_product_degrees": st["split_k3"] if args.precision == "bf16x3" else None},
        "gram": {"TFLOPs": gram_flops / (st["ms_gram"] * 1e-3) / 1e12,
                 "frac_mfma_fp64": gram_flops / (st["ms_gram"] * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["fp64"]},
        "phases_ms": phases,
        "roofline": roof,
    }

    comparisons = {}
    if not args.no_fp64 and args.precision != "fp64":
        ms64, dos64, *_ = run("fp64", 1, 1, budget=budget_left())
        l1 = float(np.abs(dos - dos64).sum() / np.abs(dos64).sum())
        comparisons["fp64"] = {"s_per_dos": ms64 / 1e3, "speedup_of_measured_path": ms64 / ms,
                               "dos_l1_measured_vs_fp64": l1}
        if not args.no_bf16:
            for other in ("fp32", "bf16x3", "bf16"):
                if other == args.precision:
                    continue
                mso, doso, *_ = run(other, 1, 1, budget=0)
                comparisons[other] = {"s_per_dos": mso / 1e3,
                                      "dos_l1_vs_fp64": float(np.abs(doso - dos64).sum() / np.abs(dos64).sum())}
    if not args.no_dgc:
        # Algorithm 2 on the same recurrence: the moments ride on the steps s <= M/2
        msd, dosd, _, _, std = run(args.precision, 1, 1, budget=0, dgc=True)
        keep = dos > 1e-2 * dos.max()
        comparisons["dgc_by_product"] = {
            "s_per_dos": msd / 1e3, "ms_recurrence": std["ms_recurrence"],
            "ms_recurrence_without": st["ms_recurrence"],
            "ssm_dos_max_rel_change": float(np.abs(dosd - dos).max() / dos.max()),
            "dgc_vs_ssm_l1_resolved": float(np.abs(dgc_out["dos"][keep] - dosd[keep]).sum() / np.abs(dosd[keep]).sum())}
    if not args.no_ress:
        # Algorithm 7 on the same workload: N_v = 80 alone, and 40 + 40 with the hybrid
        # correction of Algorithm 6 (the paper's split when N_v is short of the rank); the
        # recurrence in FP64, and in FP32 for the split
        keep = dos > 1e-2 * dos.max()
        for rprec, nvr, nvh in (("fp64", 80, 0), ("fp64", 40, 40), ("fp32", 40, 40)):
            csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float64 if rprec == "fp64" else torch.float32, device=dev)
            ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nvr, degree=m, t=wl.t, precision=rprec,
                        seed=wl.seed, method="ress", nv_hybrid=nvh, budget=budget_left(), lattice=wl.lattice,
                        device=dev)
            ctx.dos()
            torch.cuda.synchronize()
            t_r = time.perf_counter()
            dres, _, _ = ctx.dos()
            torch.cuda.synchronize()
            msr = (time.perf_counter() - t_r) * 1e3
            str_ = ctx.stats()
            ctx.close()
            del ctx, csr
            torch.cuda.empty_cache()
            entry = {"s_per_dos": msr / 1e3, "phases_ms": {k: str_[k] for k in
                                                           ("ms_recurrence", "ms_gram", "ms_sweep", "ms_geneig")},
                     "ring_slots": str_["chunk"]}
            if "dos" in dgc_out:
                entry["l1_vs_dgc_resolved"] = float(np.abs(dres[keep] - dgc_out["dos"][keep]).sum()
                                                    / np.abs(dgc_out["dos"][keep]).sum())
            comparisons[f"ress_dgc_{rprec}_nv{nvr}_hybrid{nvh}"] = entry
            log(f"RESS-DGC {rprec} N_v={nvr} N~_v={nvh}: {msr:.1f} ms/DOS  phases {entry['phases_ms']}")
    out["comparisons"] = comparisons
    if adjoint:
        out["adjoint"] = adjoint
    if not args.no_large:
        out["large"] = large_workloads(S, WL, torch, dev, budget_left)
    if not args.no_large:
        out["geneig"] = geneig_scaling(S, torch, dev)
        out["small"] = small_workload(S, WL, torch, dev, oracle_small)
        out["machine"] = machine_rates(torch, dev)
        log(f"32^2 workload: {out['small']}; machine: {out['machine']}")
    if baseline is not None:
        out["cpu_baseline"] = baseline
    print(json.dumps(out), flush=True)


def stencil27_recurrence(S, WL, torch, dev, budget):
    """The 27-point 128^3 lattice (N_v = 256) at degree 400 and eight sweep points: two ssm_dos
    calls, the second's recurrence timed (us per step, GB/s on compulsory bytes)."""
    wl = WL.make_workload(5, degree=400)
    t = wl.t[wl.nt // 16::wl.nt // 8]
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=dev)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=t, precision="bf16x3",
                seed=wl.seed, budget=budget, lattice=wl.lattice, device=dev)
    ctx.dos()
    ctx.dos()
    st = ctx.stats()
    ctx.close()
    del ctx, csr
    torch.cuda.empty_cache()
    comp, _ = spmm_bytes_models(wl.a.n, wl.a.nnz, wl.nv, 4)
    us = st["ms_recurrence"] * 1e3 / st["spmm_launches"]
    out = {"workload": wl.name, "n": wl.a.n, "nnz": wl.a.nnz, "nv": wl.nv,
           "kernel": "box_step_kernel" if st["box_stencil"] else "cheb_step_kernel",
           "steps": st["spmm_launches"], "us_per_step": us, "bytes_compulsory": comp,
           "GBps_compulsory": comp / (us * 1e-6) / 1e9,
           "frac_hbm": comp / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS}
    log(f"27-point recurrence: {us:.0f} us per step, {out['GBps_compulsory']:.0f} GB/s")
    return out


def large_workloads(S, WL, torch, dev, budget_left):
    """The random-graph workload's whole DOS (split-BF16 sweep, sweep-point batches as
    planned in the free memory; its DOS against the stored oracle values when present), and
    by RESS-DGC with an FP32 recurrence; the 27-point workload's recurrence rate (N_v = 256,
    a run of 400 steps on 8 points) and its whole DOS by RESS-DGC (FP32 recurrence)."""
    res = {}
    wl = WL.make_workload(3)
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=dev)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t, precision="bf16x3",
                seed=wl.seed, budget=budget_left(12), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.reset()
    dos, r1, r2 = ctx.dos()
    s_dos = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    del ctx, csr
    torch.cuda.empty_cache()
    comp, gath = spmm_bytes_models(wl.a.n, wl.a.nnz, wl.nv, 4)
    us = st["ms_recurrence"] * 1e3 / st["spmm_launches"]
    entry = {"workload": wl.name, "n": wl.a.n, "nnz": wl.a.nnz, "nv": wl.nv, "degree": wl.degree, "nt": wl.nt,
             "precision": "bf16x3", "s_per_dos": s_dos,
             "plan": {"passes": st["passes"], "chunk": st["chunk"], "batch": st["batch"]},
             "phases_ms": {k: st[k] for k in ("ms_recurrence", "ms_sweep", "ms_gram", "ms_geneig")},
             "spmm_us_per_step": us, "spmm_GBps_compulsory": comp / (us * 1e-6) / 1e9,
             "spmm_GBps_gather_inclusive": gath / (us * 1e-6) / 1e9}
    golden = os.path.join(ROOT, "tests", "golden", "er_graph_2p20_fp64_oracle.json")
    if os.path.exists(golden):
        with open(golden) as fh:
            g = json.load(fh)
        pts, ref = np.array(g["points"]), np.array(g["dos"])
        entry["dos_l1_vs_oracle_points"] = float(np.abs(dos[pts] - ref).sum() / np.abs(ref).sum())
    res["random_graph_dos"] = entry
    log(f"random graph: {s_dos:.2f} s per DOS, plan {entry['plan']}, {us:.0f} us per step")
    # the same workload by RESS-DGC (Algorithm 7, FP32 recurrence to degree M/2 + 1): no Z,
    # so no replays of the recurrence
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=dev)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t, precision="fp32",
                seed=wl.seed, method="ress", budget=budget_left(12), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.reset()
    dres, _, _ = ctx.dos()
    s_res = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    del ctx, csr
    torch.cuda.empty_cache()
    res["random_graph_ress_dgc_fp32"] = {
        "s_per_dos": s_res, "ring_slots": st["chunk"], "steps": st["spmm_launches"],
        "phases_ms": {"recurrence": st["ms_recurrence"], "pair_gram": st["ms_gram"],
                      "moments_and_sums": st["ms_sweep"], "geneig": st["ms_geneig"]}}
    log(f"random graph, RESS-DGC FP32: {s_res:.2f} s per DOS")

    res["stencil27_recurrence"] = stencil27_recurrence(S, WL, torch, dev, budget_left(12))
    # its whole DOS (M = 4000, N_t = 4000) by RESS-DGC with an FP32 recurrence: SS-DGC would
    # need about 36 sweep-point batches, each replaying the 4000 steps
    wl = WL.make_workload(5)
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=dev)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t, precision="fp32",
                seed=wl.seed, method="ress", budget=budget_left(12), lattice=wl.lattice, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.reset()
    ctx.dos()
    s_res = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    del ctx, csr
    torch.cuda.empty_cache()
    res["stencil27_ress_dgc_fp32"] = {
        "workload": wl.name, "nv": wl.nv, "degree": wl.degree, "nt": wl.nt, "s_per_dos": s_res,
        "ring_slots": st["chunk"], "steps": st["spmm_launches"],
        "phases_ms": {"recurrence": st["ms_recurrence"], "pair_gram": st["ms_gram"],
                      "moments_and_sums": st["ms_sweep"], "geneig": st["ms_geneig"]}}
    log(f"27-point workload, RESS-DGC FP32: {s_res:.1f} s per DOS")
    return res


if __name__ == "__main__":
    main()
