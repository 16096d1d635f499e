"""Full-size parity for the other workloads, in the planner's own launch configuration:

* er_graph_laplacian_2p20_deg16 (N = 2^20, nnz 17.8M, N_v = 128, M = 2000) and
  stencil27_128cube_lognormal (N = 2^21, nnz 56.6M, N_v = 256, M = 4000): the oracle
  cannot run these in a test (hours on the host), so a strided subset of the sweep
  points runs at full N, N_v and M, and the oracle checks sampled outputs one by one:
  Chebyshev steps of the last ring chunk on sampled rows, sampled entries of the Gram
  matrices, and Algorithm 4 on every point from the device's Gram matrices; the DOS
  obeys 0 <= phi <= N_v (1 + rho) g_max and r2 <= r1 <= N_v.
* anderson3d_64cube_W4_shifted_spd (N = 262144, N_v = 80, M = 1500, N_t = 1500): the
  FP32 and split-BF16 DOS against stored oracle values at ten strided points
  (tests/golden/anderson64_spd_fp64_oracle.json, written by make_golden.py from the
  oracle only), and the adjoint with checkpoints every 50 degrees against the resident
  adjoint and central differences.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import ssm_oracle as O
from paper_1504_07690_amd import workloads as WL

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "anderson64_spd_fp64_oracle.json")
GOLDEN3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "er_graph_2p20_fp64_oracle.json")


@pytest.fixture(scope="module")
def S():
    from paper_1504_07690_amd import ssm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ssm


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _budget(reserve_gib=24):
    _free()
    free, _ = torch.cuda.mem_get_info()
    return int(free - reserve_gib * (1 << 30))


def _ctx(S, wl, precision, t, budget=0, ckpt_every=0):
    dt = torch.float64 if precision == "fp64" else torch.float32
    csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=t, precision=precision,
                seed=wl.seed, budget=budget, ckpt_every=ckpt_every, lattice=wl.lattice, device=DEV)
    return csr, ctx


def _check_sampled_stages(wl, ctx, t, dos, r1, r2, rng):
    """Stage outputs of a finished ssm_dos against the oracle's arithmetic, sampled."""
    a = wl.a
    n, nv, m = a.n, wl.nv, wl.degree
    v = ctx.views()
    chunk = v["chunk"]
    y = v["y"]
    alpha = 2.0 / (wl.hi - wl.lo)
    beta = -(wl.hi + wl.lo) / (wl.hi - wl.lo)
    gmax = O.range_bound(wl.sigma, n)
    # invariants of the estimate
    assert np.all(np.isfinite(dos)) and np.all(dos >= 0) and np.all(dos <= nv * (1 + 1e-3) * gmax)
    assert np.all(r2 <= r1) and np.all(r1 <= nv)
    # (1) Chebyshev steps at the end of the recurrence, on sampled rows: the ring's last
    # writes hold Y_{M-3} .. Y_M whenever it has at least 4 slots
    ks = [m, m - 1] if chunk >= 4 else [m]
    rows = rng.integers(0, n, 5)
    for k in sorted(set(ks)):
        for r in rows:
            cols = a.col_idx[a.row_ptr[r]:a.row_ptr[r + 1]]
            vals = a.values[a.row_ptr[r]:a.row_ptr[r + 1]]
            ym1 = y[(k - 1) % chunk][torch.as_tensor(cols, device=DEV)].double().cpu().numpy()
            ym1_r = y[(k - 1) % chunk][int(r)].double().cpu().numpy()
            ym2_r = y[(k - 2) % chunk][int(r)].double().cpu().numpy()
            pred = 2 * (alpha * (vals @ ym1) + beta * ym1_r) - ym2_r
            got = y[k % chunk][int(r)].double().cpu().numpy()
            mag = 2 * (alpha * (np.abs(vals) @ np.abs(ym1)) + abs(beta) * np.abs(ym1_r)) + np.abs(ym2_r)
            assert np.all(np.abs(got - pred) <= 64 * 2.0 ** -24 * mag + 1e-30), (k, r)
    # (2) sampled Gram entries of two points against the oracle's K_Z = Z^T Z and
    # K_W = (W^T Z + Z^T W)/2; the kernel forms only the upper 16 x 16 blocks of W^T Z, so K_W
    # may also differ by half the asymmetry |w_p . z_q - w_q . z_p| / 2 of the rounded Z
    z = v["z"]
    w = v["w"]
    for i in (0, len(t) - 1):
        for (p, q) in ((0, 0), (0, nv - 1), (nv // 2, nv // 3), (nv - 1, nv - 1)):
            zi = z[i][:, [p, q]].double().cpu().numpy()
            wi = w[:, [p, q]].double().cpu().numpy()
            zp, zq = zi[:, 0], zi[:, 1]
            wp, wq = wi[:, 0], wi[:, 1]
            tol = (n + 4) * 2.0 ** -53
            kz = v["k_z"][i, p, q].item()
            kw = v["k_w"][i, p, q].item()
            assert abs(kz - zp @ zq) <= tol * (np.abs(zp) @ np.abs(zq)) + 1e-300
            ref_w = 0.5 * (wp @ zq + wq @ zp)
            mag_w = 0.5 * (np.abs(wp) @ np.abs(zq) + np.abs(wq) @ np.abs(zp))
            asym = 0.5 * abs(wp @ zq - wq @ zp)
            assert abs(kw - ref_w) <= tol * mag_w + asym + 1e-300
    # (3) Algorithm 4 on every point from the device's Gram matrices
    kw = v["k_w"].cpu().numpy()
    kz = v["k_z"].cpu().numpy()
    fl = _floors(wl, ctx, v, t)
    ref = np.array([O.geneig_trace(kw[i], kz[i], gmax, s_floor=fl[i])[0] for i in range(len(t))])
    bad = np.abs(dos - ref) > 1e-9 * gmax
    assert bad.sum() <= 1, np.nonzero(bad)
    # (4) where the plan keeps every block: rows of Z against the oracle's sweep of the
    # device's own blocks
    if chunk == m + 1 and v["batch"] == len(t):
        rows_t = torch.as_tensor(rng.integers(0, n, 4), device=DEV)
        yr = y[:, rows_t, :].double().cpu().numpy()
        zr = z[:, rows_t, :].double().cpu().numpy()
        mu = O.dgc_coefficients(t, m, wl.sigma, n, wl.lo, wl.hi)
        _assert_z_rows(zr, mu, yr, ctx.precision, ctx.stats()["split_k3"])


ETA = {"fp64": 0.0, "fp32": 2.0 ** -22, "bf16x3": 2.0 ** -16, "bf16": 2.0 ** -7}


def _floors(wl, ctx, v, t):
    """The rounding floors of Algorithm 4's truncation that the device used, checked against
    the oracle's formula eta ||mu(t_i)||_2 ||W||_F^2 / sqrt(N N_v) on the device's W."""
    eta = ETA[ctx.precision]
    if eta == 0.0:
        assert "s_floor" not in v
        return np.zeros(len(t))
    fl = v["s_floor"].cpu().numpy()
    wsq = float(torch.sum(v["w"].double() ** 2).item())
    mu = O.dgc_coefficients(t, wl.degree, wl.sigma, wl.a.n, wl.lo, wl.hi)
    ref = eta * np.sqrt((mu ** 2).sum(axis=0)) * wsq / np.sqrt(wl.a.n * wl.nv)
    assert np.allclose(fl, ref, rtol=1e-9, atol=0)
    return fl


def _assert_z_rows(zr, mu, yr, precision, k3):
    """Rows of Z (points x rows x N_v) against the oracle's sweep (Algorithm 5 steps 6-8)
    of the same rows of the device's blocks yr ((M+1) x rows x N_v), within the rounding
    bound of the sweep's arithmetic: FP32 products and sums; for split BF16 at most
    2^-16 |mu||y| per term below k3 (three products, each operand carried to 2^-17) and
    2^-7 |mu||y| past it (one product of two 8-bit operands), plus the FP32 sums."""
    kk = mu.shape[0]
    pred = O.sweep(mu, iter(yr))
    mag = O.sweep(np.abs(mu), iter(np.abs(yr)))
    sums = (kk + 3) * 2.0 ** -24 * mag
    if precision == "bf16x3":
        k3 = max(0, min(k3, kk))
        lead = O.sweep(np.abs(mu[:k3]), iter(np.abs(yr[:k3]))) if k3 else 0.0
        tail = O.sweep(np.abs(mu[k3:]), iter(np.abs(yr[k3:]))) if k3 < kk else 0.0
        tol = 2.0 ** -16 * lead + 2.0 ** -7 * tail + sums
    elif precision == "fp32":
        tol = sums
    else:
        tol = 2.0 ** -7 * mag + sums  # plain BF16 operands
    err = np.abs(zr - pred)
    assert np.all(err <= tol + 1e-30), float((err / (tol + 1e-30)).max())


@pytest.mark.parametrize("cfg,degree", [(3, 64), (5, 32)])
def test_large_split_sweep_z_rows(S, cfg, degree):
    """The split-BF16 sweep where N N_v is so large (28 N N_v + 1024 >= 2^31) that each degree
    of Y takes its own buffer resource: the random-graph and 27-point workloads at full N and
    N_v with a reduced degree, eight strided sweep points.  Rows of Z against the oracle's
    sweep of the device's own blocks, first with every block resident (one sweep launch),
    then with a ring of fewer blocks (launches from mid-table degrees that accumulate into
    Z); the recurrence is deterministic, so both runs see the same blocks."""
    wl = WL.make_workload(cfg, degree=degree)
    n, nv, m = wl.a.n, wl.nv, degree
    assert 28 * n * nv + 1024 >= 2 ** 31
    t = wl.t[wl.nt // 16::wl.nt // 8]
    rng = np.random.default_rng(100 + cfg)
    rows_t = torch.as_tensor(np.sort(rng.choice(n, 6, replace=False)), device=DEV)
    mu = O.dgc_coefficients(t, m, wl.sigma, n, wl.lo, wl.hi)
    csr, ctx = _ctx(S, wl, "bf16x3", t)
    st = ctx.stats()
    assert st["passes"] == 1 and st["chunk"] == m + 1, st
    dos1, r1, r2 = ctx.dos()
    v = ctx.views()
    yr = v["y"][:, rows_t, :].double().cpu().numpy()
    z1 = v["z"][:, rows_t, :].double().cpu().numpy()
    k3 = ctx.stats()["split_k3"]
    full = S.workspace_size(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=m, nt=len(t),
                            precision="bf16x3", seed=wl.seed, lattice=wl.lattice)
    ctx.close()
    del ctx, v
    _free()
    print(f"{wl.name} M={m}: resident plan, k3 {k3}, DOS max {dos1.max():.3e}")
    _assert_z_rows(z1, mu, yr, "bf16x3", k3)
    # a ring of fewer blocks: launches start at degrees that are multiples of 16 and add into Z
    e_bytes = n * nv * 4
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=m, t=t, precision="bf16x3",
                seed=wl.seed, budget=full - 17 * e_bytes, lattice=wl.lattice, device=DEV)
    st = ctx.stats()
    assert st["passes"] == 1 and 16 <= st["chunk"] < m + 1 and st["chunk"] % 16 == 0, st
    dos2, _, _ = ctx.dos()
    st = ctx.stats()
    assert st["sweep_launches"] == -(-(m + 1) // st["chunk"])
    v = ctx.views()
    k_first = (m // st["chunk"]) * st["chunk"]
    y_last = v["y"][:, rows_t, :].double().cpu().numpy()
    for k in range(k_first, m + 1):  # the ring's last blocks are the resident run's
        assert np.array_equal(y_last[k % st["chunk"]], yr[k]), k
    z2 = v["z"][:, rows_t, :].double().cpu().numpy()
    ctx.close()
    del ctx, v, csr
    _free()
    print(f"ring {st['chunk']}: {st['sweep_launches']} sweep launches; DOS L1 vs the resident plan "
          f"{np.abs(dos2 - dos1).sum() / np.abs(dos1).sum():.2e}")
    _assert_z_rows(z2, mu, yr, "bf16x3", k3)
    assert np.abs(dos2 - dos1).sum() <= 1e-3 * np.abs(dos1).sum()


@pytest.mark.parametrize("cfg,precision", [(3, "bf16x3"), (3, "bf16"), (5, "bf16x3")])
def test_large_workload_sampled_stages(S, cfg, precision):
    wl = WL.make_workload(cfg)
    t = wl.t[wl.nt // 16::wl.nt // 8]  # 8 strided sweep points
    csr, ctx = _ctx(S, wl, precision, t, budget=_budget())
    try:
        dos, r1, r2 = ctx.dos()
        st = ctx.stats()
        print(f"{wl.name} {precision}: plan {st['passes']} pass(es), ring {st['chunk']}, "
              f"{st['ms_total']:.0f} ms (recurrence {st['ms_recurrence']:.0f}, sweep {st['ms_sweep']:.0f}, "
              f"Gram {st['ms_gram']:.0f}, Alg. 4 {st['ms_geneig']:.0f}); r1 {r1.tolist()}")
        _check_sampled_stages(wl, ctx, t, dos, r1, r2, np.random.default_rng(cfg))
    finally:
        ctx.close()
        del ctx, csr
        _free()



def test_random_graph_dos_against_stored_oracle(S):
    """The random-graph workload's whole DOS (N = 2^20, N_v = 128, M = 2000, N_t = 2000,
    split-BF16 sweep, sweep-point batches as planned in the free memory) against the
    oracle's FP64 SS-DGC at 16 strided points on the same W: relative L1 within 1e-3 (the
    kept ranks are printed beside the oracle's)."""
    if not os.path.exists(GOLDEN3):
        pytest.skip("stored oracle values of the random-graph workload are not present")
    with open(GOLDEN3) as fh:
        g = json.load(fh)
    wl = WL.make_workload(3)
    assert wl.a.n == g["n"] and wl.a.nnz == g["nnz"] and abs(wl.lo - g["lo"]) < 1e-12
    csr, ctx = _ctx(S, wl, "bf16x3", wl.t, budget=_budget())
    dos, r1, r2 = ctx.dos()
    st = ctx.stats()
    ctx.close()
    del ctx, csr
    _free()
    pts, ref = np.array(g["points"]), np.array(g["dos"])
    l1 = np.abs(dos[pts] - ref).sum() / np.abs(ref).sum()
    print(f"{wl.name} bf16x3: plan {st['passes']} pass(es), ring {st['chunk']}, {st['ms_total'] / 1e3:.1f} s; "
          f"L1 vs the stored oracle values at {len(pts)} points {l1:.2e}; r1 {r1[pts].tolist()} "
          f"(oracle {g['r1']})")
    assert l1 <= 1e-3


def test_random_graph_ress_dgc_full_size(S):
    """RESS-DGC (Algorithm 7) on the random-graph workload at full size (N = 2^20, N_v = 128,
    M = 2000, N_t = 2000: 1001 recurrence steps, no Z), with an FP32 and an FP64 recurrence:
    the moments X_0..X_2 of the device's block against the oracle's W^T T_l(A~) W on the same
    W, the DOS within 0 <= phi <= N_v (1 + rho) g_max, and the FP32 path's DOS within 1e-3
    relative L1 of the FP64 path's."""
    wl = WL.make_workload(3)
    g_max = O.range_bound(wl.sigma, wl.a.n)
    out = {}
    for precision in ("fp64", "fp32"):
        dt = torch.float64 if precision == "fp64" else torch.float32
        csr = S.DeviceCSR.from_csr(wl.a, dtype=dt, device=DEV)
        ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t,
                    precision=precision, seed=wl.seed, method="ress", budget=_budget(), device=DEV)
        dos, r1, r2 = ctx.dos()
        st = ctx.stats()
        v = ctx.views()
        x = v["moments"][:3].cpu().numpy()
        w = v["w"].double().cpu().numpy()
        ctx.close()
        del ctx, csr, v
        _free()
        print(f"{wl.name} RESS-DGC {precision}: {st['ms_total'] / 1e3:.2f} s (recurrence {st['ms_recurrence']:.0f}, "
              f"pair Gram {st['ms_gram']:.0f}, moments {st['ms_sweep']:.0f}, Alg. 4 {st['ms_geneig']:.0f} ms), "
              f"ring {st['chunk']}, r1 {r1.min()}..{r1.max()}")
        ref = np.zeros_like(x)
        for l, v_c in O.chebyshev_blocks(wl.a, w, 2, wl.lo, wl.hi):
            ref[l] = w.T @ v_c
        err = np.abs(x - ref).max() / np.abs(ref[0]).max()
        print(f"  moments X_0..X_2: max error {err:.2e} of max|X_0|")
        assert err <= (1e-11 if precision == "fp64" else 1e-5)
        assert np.all(np.isfinite(dos)) and dos.min() >= 0.0 and dos.max() <= wl.nv * (1 + 1e-3) * g_max
        out[precision] = dos
    l1 = np.abs(out["fp32"] - out["fp64"]).sum() / np.abs(out["fp64"]).sum()
    print(f"  FP32 against FP64 recurrence: DOS L1 {l1:.2e}")
    assert l1 <= 1e-3


@pytest.fixture(scope="module")
def golden4():
    if not os.path.exists(GOLDEN4):
        pytest.skip("stored oracle values of the shifted SPD workload are not present")
    with open(GOLDEN4) as fh:
        return json.load(fh)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_spd_workload_against_stored_oracle(S, golden4, precision):
    g = golden4
    wl = WL.make_workload(4)
    assert wl.a.n == g["n"] and wl.a.nnz == g["nnz"] and abs(wl.lo - g["lo"]) < 1e-12
    csr, ctx = _ctx(S, wl, precision, wl.t)
    dos, r1, r2 = ctx.dos()
    ctx.close()
    del ctx, csr
    _free()
    pts = np.array(g["points"])
    ref = np.array(g["dos"])
    l1 = np.abs(dos[pts] - ref).sum() / np.abs(ref).sum()
    # Tr log(A) at full size (Algorithm 8, f floored at half the Gershgorin bound 0.1): the
    # library's weights against the oracle's, the weighted sum over the stored points
    # against the oracle's, and the whole trace (reported: the oracle's DOS is stored at ten
    # points only, and sigma^ = 1/150 lies past the deconvolution's well-posed range)
    f = lambda x: np.log(np.maximum(x, 0.05))
    w_dev = S.trace_weights(lambda x: float(f(x)), lo=wl.lo, hi=wl.hi, nt=wl.nt, n=wl.a.n, sigma=wl.sigma)
    w_or = O.trace_weights(f, wl.a.n, wl.lo, wl.hi, wl.nt, wl.sigma)
    assert np.abs(w_dev - w_or).max() <= 1e-9 * np.abs(w_or).max()
    part_dev, part_or = float(w_dev[pts] @ dos[pts]), float(w_or[pts] @ ref)
    print(f"shifted SPD {precision}: L1 vs the stored oracle values {l1:.2e}; Tr log(A) over the stored points "
          f"{part_dev:.10e} (oracle {part_or:.10e}, rel {abs(part_dev - part_or) / abs(part_or):.2e}); whole "
          f"Tr log(A) = {float(w_dev @ dos):.8e}")
    assert l1 <= 1e-3
    assert abs(part_dev - part_or) <= 1e-3 * abs(part_or)


def test_spd_workload_checkpointed_adjoint(S):
    """The adjoint with checkpoints every 50 degrees, as the workload asks: equal to the
    resident adjoint up to the rounding of the chunked forward sweep, and along a
    symmetric direction close to central differences of the FP32 DOS."""
    from test_oracle_pins import _sym_direction
    wl = WL.make_workload(4)
    csr, ctx = _ctx(S, wl, "fp32", wl.t)
    dos, _, _ = ctx.dos()
    dos_bar = np.random.default_rng(9).uniform(0.0, 1.0, wl.nt) * (dos > 1e-2 * dos.max())
    g_res = ctx.backward(dos_bar).cpu().numpy()
    ctx.close()
    del ctx, csr
    _free()
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=DEV)
    ctx = S.SSM(csr, lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=wl.nv, degree=wl.degree, t=wl.t, precision="fp32",
                seed=wl.seed, ckpt_every=50, plan=(wl.nt, 208), device=DEV)
    st = ctx.stats()
    assert st["passes"] == 1 and 50 <= st["chunk"] < wl.degree + 1, st
    ctx.dos()
    g = ctx.backward(dos_bar).cpu().numpy()
    bs = ctx.backward_stats()
    rel = np.linalg.norm(g - g_res) / np.linalg.norm(g_res)
    print(f"shifted SPD adjoint: ring {st['chunk']}, {bs['segments']} segments, {bs['recomputed']} blocks "
          f"recomputed, {bs['ms_total']:.0f} ms; vs resident {rel:.2e}")
    assert rel <= 1e-3
    base = csr.values.clone()
    h = 1e-3 * np.abs(wl.a.values).max()
    ed = torch.tensor(_sym_direction(wl.a, 0), dtype=torch.float32, device=DEV)
    csr.values.copy_(base + h * ed)
    lp, p1, p2 = ctx.dos()
    csr.values.copy_(base - h * ed)
    lm, m1, m2 = ctx.dos()
    csr.values.copy_(base)
    keep = dos_bar != 0
    fd = dos_bar @ (lp - lm) / (2 * h)
    ad = g @ ed.double().cpu().numpy()
    print(f"direction 0: adjoint {ad:.6e}  central difference (FP32 DOS) {fd:.6e}; kept sets "
          f"{'unchanged' if np.array_equal(p1[keep], m1[keep]) and np.array_equal(p2[keep], m2[keep]) else 'changed'}")
    if np.array_equal(p1[keep], m1[keep]) and np.array_equal(p2[keep], m2[keep]):
        assert abs(ad - fd) <= 1e-2 * abs(fd)
    ctx.close()
    del ctx, csr
    _free()


def _sym_hash_direction(a, seed):
    """A symmetric direction on the pattern of a (the value of entry (r, c) equals that of
    (c, r)), from a multiplicative hash of the unordered pair: vectorised for large nnz."""
    rows = np.repeat(np.arange(a.n, dtype=np.int64), np.diff(a.row_ptr))
    cols = a.col_idx.astype(np.int64)
    key = np.minimum(rows, cols) * a.n + np.maximum(rows, cols) + seed * 0x9E3779B1
    h = (key * 0x2545F491) & 0xFFFFFFFF
    h = (h ^ (h >> 15)) * 0x2C1B3C6D & 0xFFFFFFFF
    return (h ^ (h >> 12)).astype(np.float64) / 2.0 ** 32 - 0.5


def test_stencil27_adjoint_two_level_checkpoints(S):
    """The adjoint at the 27-point workload's full size (N = 128^3, N_v = 256, M = 4000,
    FP32), on eight strided sweep points: checkpoint pairs every 250 degrees and a ring of
    16 blocks, so that the backward recomputes each segment through a second level of pairs
    (one level of checkpoints would need more than the GPU's memory).  The gradient of
    sum_i dos_bar_i phi~(t_i), dos_bar weighting the resolved points, is finite and matches a
    central difference of the device's FP32 DOS along one symmetric direction (step
    1e-3 max|a|, tolerance 1e-2: the FP32 estimate's rounding over the step)."""
    wl = WL.make_workload(5)
    n, nv, m = wl.a.n, wl.nv, wl.degree
    t = wl.t[wl.nt // 16::wl.nt // 8]
    s, ring = 250, 16
    bb = n * nv * 4
    csr = S.DeviceCSR.from_csr(wl.a, dtype=torch.float32, device=DEV)
    kw = dict(lo=wl.lo, hi=wl.hi, sigma=wl.sigma, nv=nv, degree=m, precision="fp32", seed=wl.seed)
    ctx = S.SSM(csr, t=t, ckpt_every=s, plan=(len(t), ring), lattice=wl.lattice, device=DEV, **kw)
    st = ctx.stats()
    assert st["passes"] == 1 and st["chunk"] == ring, st
    dos, r1, r2 = ctx.dos()
    keep = dos > 1e-2 * dos.max()
    assert keep.sum() >= 2
    dos_bar = np.random.default_rng(11).uniform(0.5, 1.0, len(t)) * keep
    g = ctx.backward(dos_bar)
    bs = ctx.backward_stats()
    print(f"{wl.name} adjoint: ring {st['chunk']}, checkpoints every {s}: levels {bs['levels']}, "
          f"{bs['recomputed']} blocks recomputed; {bs['ms_total'] / 1e3:.1f} s (recompute "
          f"{bs['ms_recompute'] / 1e3:.1f}, reverse {bs['ms_reverse'] / 1e3:.1f}, Ybar {bs['ms_ybar'] / 1e3:.1f})")
    assert bs["levels"] == 2 and bs["recomputed"] > m
    assert bool(torch.isfinite(g).all().item())
    g = g.cpu().numpy()
    e = _sym_hash_direction(wl.a, 1)
    h = 1e-3 * np.abs(wl.a.values).max()
    base = csr.values.clone()
    ed = torch.tensor(e, dtype=torch.float32, device=DEV)
    csr.values.copy_(base + h * ed)
    lp, p1, p2 = ctx.dos()
    csr.values.copy_(base - h * ed)
    lm, q1, q2 = ctx.dos()
    csr.values.copy_(base)
    ctx.close()
    del ctx, csr, base, ed
    _free()
    same = np.array_equal(p1[keep], q1[keep]) and np.array_equal(p2[keep], q2[keep])
    fd = dos_bar @ (lp - lm) / (2 * h)
    ad = g @ e
    print(f"direction: adjoint {ad:.6e}  central difference {fd:.6e}  rel {abs(ad - fd) / abs(fd):.2e}; kept sets "
          f"{'unchanged' if same else 'changed'}")
    assert same
    assert abs(ad - fd) <= 1e-2 * abs(fd)
