#!/usr/bin/env python
"""BSPAI-GMRES-IR on one MI355X: solves/s and bucketed M-apply bandwidth.

A step is one full gmres_ir_solve (Algorithm 4 after the SPAI build: x_0,
refinement residuals in double-double, left-preconditioned MGS-GMRES with the
bucketed SPAI applied in FP32, updates) on the 256 x 256 upwind
convection-diffusion system (n = 65,536, Peclet 50), SPAI on the pattern of
A^2 built in FP64, buckets {fp64, fp32, fp16, bf16} at eps_b = 1e-4,
b = A x_true.  A, M and b are resident on the GPU before timing starts.

Printed (one JSON line): solves/s, the solver kernel's roofline (algorithmic
bytes / kernel time measured with HIP events on its stream), the CPU oracle
timed on the host, the all-FP64 SPAI-GMRES-IR comparator at equal stopping
tolerance, and the bucketed apply's HBM bandwidth on a cold 2.1M-row operator.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
VALUE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 1, 5: 0}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve_bytes(stats, n, nnz_a, mstats, vt_bytes=4, x0_fp64_nnz=None):
    """Algorithmic HBM bytes of one gmres_ir_solve (each array touched once per use).

    Per GMRES iteration j (0-based): A_p v (vt nnz + 4 nnz + 4 (n+1) + 2 vt n),
    M_b w (sum_k nnz_k (b_k + 4) + 4 (n+1) per stored bucket + 2 vt n), MGS
    reads v_0..v_j and z and writes v_{j+1}: (j + 3) vt n.  Per correction:
    residual 12 nnz + 4 (n+1) + 16 n (A in FP64 with columns, b, x) + vt n,
    s = M_b r, d = V y (its vt n) and x += d (16 n).  Start: ||A|| (12 nnz),
    x_0 = M b with the FP64 M (12 nnz_M + 16 n + 4 (n+1)).
    """
    rp = 4 * (n + 1)
    mb = sum(c * (VALUE_BYTES[p] + 4) for c, p in zip(mstats["count"], mstats["precs"]) if p != 5)
    mb += rp * sum(1 for c, p in zip(mstats["count"], mstats["precs"]) if c > 0 and p != 5) + 2 * vt_bytes * n
    ap = (vt_bytes + 4) * nnz_a + rp + 2 * vt_bytes * n
    total = 12 * nnz_a + rp
    nnz_m = x0_fp64_nnz if x0_fp64_nnz is not None else sum(mstats["count"])
    total += 12 * nnz_m + rp + 16 * n
    for its in stats["its"]:
        total += 12 * nnz_a + rp + 16 * n + vt_bytes * n  # residual
        total += mb  # s = M_b r
        for j in range(its):
            total += ap + mb + (j + 3) * vt_bytes * n
        total += its * vt_bytes * n + 16 * n
    total += 12 * nnz_a + rp + 16 * n  # final residual
    return total


def _emit(B, torch, obj):
    """Release the solver's cached workspace, then print the JSON line."""
    B.release_workspace()
    torch.cuda.synchronize()
    print(json.dumps(obj), flush=True)


def _src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src, record="solve_kernel_traffic.json"):
    """HBM traffic per launch from the committed rocprofv3 counter runs, only if
    they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", record)
    try:
        with open(p) as f:
            t = json.load(f)
        if t.get("source_sha256_16") == _src_hash(kernel_src):
            return t.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--gmres-max", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-apply-bench", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-RHS and the 32-system measurements")
    ap.add_argument("--only-apply", action="store_true", help="run only the cold bucketed-apply measurement")
    ap.add_argument("--only-batched", action="store_true", help="run only the 64-RHS measurement")
    ap.add_argument("--only-multi", action="store_true", help="run only the 32-system measurement")
    ap.add_argument("--only-powerlaw", action="store_true", help="run only the power-law matrix measurement")
    ap.add_argument("--only-gradient", action="store_true", help="run only the 512^2 gradient measurement")
    ap.add_argument("--only-adaptive", action="store_true", help="run only the adaptive-SPAI measurement")
    ap.add_argument("--only-bucketed-a", action="store_true", help="run only the bucketed-A measurement")
    ap.add_argument("--only-low-uf", action="store_true", help="run only the low-u_f SPAI measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy first (calibration of hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only: the solver is one persistent kernel per "
                                   "system; run with --gpus 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2307_03914_amd as B
    import workloads as W

    torch.cuda.set_device(0)
    dev = "cuda"
    if args.copy_calibration:
        # a plain device copy of known size (1 GiB read, 1 GiB written), for
        # scaling hardware byte counters
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b2 = torch.empty_like(a)
        torch.cuda.synchronize()
        b2.copy_(a)
        torch.cuda.synchronize()
        del a, b2
        torch.cuda.empty_cache()
    if args.only_apply:
        res = apply_bench(B, W, torch, np)
        _emit(B, torch, {"m_apply": res})
        return
    kw0 = dict(tau=1e-4, tol_rr=1e-10, gmres_max=args.gmres_max, i_max=20)
    if args.only_batched:
        _emit(B, torch, {"batched_rhs": batched_bench(B, W, torch, np, kw0)})
        return
    if args.only_multi:
        _emit(B, torch, {"multi_system": multi_bench(B, W, torch, np, kw0)})
        return
    if args.only_powerlaw:
        _emit(B, torch, {"powerlaw": powerlaw_bench(B, W, torch, np, kw0)})
        return
    if args.only_gradient:
        _emit(B, torch, {"gradient": gradient_bench(B, W, torch, np)})
        return
    if args.only_adaptive:
        _emit(B, torch, {"adaptive_spai": adaptive_bench(B, W, torch, np, kw0)})
        return
    if args.only_bucketed_a:
        _emit(B, torch, {"bucketed_a": bucketed_a_bench(B, W, torch, np, kw0)})
        return
    if args.only_low_uf:
        _emit(B, torch, {"low_uf_spai": low_uf_bench(B, W, torch, np, kw0)})
        return
    _log("generating workload")
    c = W.config("2")
    A, P = c["A"], c["P"]
    n = A.n
    Ad = B.CSRMatrix.from_host(A)
    Pd = B.CSRMatrix.from_host(P)
    b = torch.as_tensor(c["b"], device=dev)
    precs = c["precs"]
    kw = dict(tau=1e-4, tol_rr=1e-10, gmres_max=args.gmres_max, i_max=20)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = B.build(Ad, Pd, eps=args.eps, precs=precs)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    mst = h.stats()
    _log(f"built M: counts {mst['count']} storage {mst['storage_pct']:.1f}% in {build_ms:.1f} ms")

    for _ in range(args.warmup):
        x, st = B.solve(Ad, b, h, **kw)
    torch.cuda.synchronize()
    B.set_profiling(True)
    kernel_ms = []
    stats = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, stats = B.solve(Ad, b, h, **kw)
        kernel_ms.append(B.last_solve_kernel_ms())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.set_profiling(False)
    ms_per_step = elapsed * 1e3 / args.steps
    solves_per_s = args.steps / elapsed
    xh = x.cpu().numpy()
    fwd = float(np.abs(xh - c["x_true"]).max() / np.abs(c["x_true"]).max())
    _log(f"BSPAI: {solves_per_s:.2f} solves/s, its {stats['its']}, relres {stats['relres'][-1]:.2e}")

    kern_ms = float(np.mean(kernel_ms))
    nbytes = solve_bytes(stats, n, A.nnz, mst)
    kernel_src = os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "solve.hip")
    roofline = {"kernel": "k_gmres_ir (persistent solver)", "bound": "hbm",
                "achieved": nbytes / (kern_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": nbytes / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "traffic": _traffic(kernel_src),
                "algorithmic_bytes": nbytes, "kernel_ms": kern_ms}

    # the latency bound of the persistent solver: its dependent grid-wide
    # exchanges (each MGS pass and norm is an all-reduction, each published
    # vector a barrier) times the measured cost of one exchange
    G = B.solve_blocks(n)
    ex_us = B.exchange_latency_us(G)
    n_ex = 3 + sum(6 + sum(j + 4 for j in range(k)) for k in stats["its"])
    latency = {"blocks": G, "exchange_us": ex_us, "exchanges_per_solve": n_ex,
               "floor_ms": n_ex * ex_us * 1e-3, "frac": n_ex * ex_us * 1e-3 / kern_ms}
    _log(f"latency floor: {n_ex} exchanges x {ex_us:.2f} us = {n_ex * ex_us * 1e-3:.1f} ms "
         f"({100 * latency['frac']:.0f}% of the kernel time)")
    roofline["latency_floor"] = latency

    out = {"metric": "GMRES-IR solves/s & M-apply HBM GB/s, BSPAI vs fp64 SPAI at equal backward error",
           "value": solves_per_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"convdiff2d 256x256 upwind Pe=50 (n=65536), SPAI pattern(A^2) FP64, "
                                  f"buckets fp64/fp32/fp16/bf16 eps={args.eps:g}, u_g=u_p=fp32, u_r=double-double, "
                                  f"tau=1e-4, refine to 1e-10 rel. residual, GMRES cap {args.gmres_max}",
                      "n": n, "nnz_A": A.nnz, "nnz_M": int(sum(mst["count"])), "bucket_counts": mst["count"],
                      "storage_pct": mst["storage_pct"]},
           "solve": {"its": stats["its"], "its_total": stats["its_total"], "relres": stats["relres"][-1],
                     "eta": stats["eta"][-1], "forward_error": fwd, "build_ms": build_ms},
           "roofline": roofline}

    if not args.no_comparators:
        # all-FP64 SPAI-GMRES-IR (u_g = u_p = fp64, tau = 1e-8, one fp64 bucket) at the same stopping test,
        # and the fp64 M with FP32 Krylov (isolates the effect of bucketing)
        comps = {}
        h64 = B.build(Ad, Pd, eps=2.0 ** -53, precs=["fp64"])
        for name, hh, extra in (("spai_fp64_all", h64, dict(u_g="fp64", tau=1e-8)),
                                ("spai_fp64M_fp32krylov", h64, {}),
                                ("bspai_cgs2", h, dict(orth="cgs2"))):
            k2 = dict(kw)
            k2.update(extra)
            for _ in range(2):
                x2, s2 = B.solve(Ad, b, hh, **k2)
            reps = max(3, args.steps // 4)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                x2, s2 = B.solve(Ad, b, hh, **k2)
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            comps[name] = {"solves_per_s": reps / el, "its": s2["its"], "relres": s2["relres"][-1],
                           "eta": s2["eta"][-1]}
            _log(f"{name}: {reps / el:.2f} solves/s its {s2['its']}")
        out["comparators"] = comps
        # the workload's sweep over eps_b: occupancy, storage and iterations
        # per eps against the unbucketed fp64 SPAI (plain SPAI-GMRES-IR with
        # the same fp32 Krylov)
        sweep = []
        for eps in (1e-6, 1e-4, 1e-2):
            he = B.build(Ad, Pd, eps=eps, precs=precs)
            se = he.stats()
            B.solve(Ad, b, he, **kw)
            torch.cuda.synchronize()
            reps = 3
            t1 = time.perf_counter()
            for _ in range(reps):
                xe, ste = B.solve(Ad, b, he, **kw)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t1) / reps
            sweep.append({"eps": eps, "bucket_counts": se["count"], "storage_pct": se["storage_pct"],
                          "its": ste["its"], "its_total": ste["its_total"], "eta": ste["eta"][-1],
                          "relres": ste["relres"][-1], "solves_per_s": 1.0 / el})
            he.free()
            _log(f"eps {eps:g}: counts {se['count']} storage {se['storage_pct']:.1f}% its {ste['its']} "
                 f"{1.0 / el:.2f} solves/s")
        out["eps_sweep"] = {"plain_spai_its": comps["spai_fp64M_fp32krylov"]["its"], "points": sweep}
        h64.free()

    if not args.no_apply_bench:
        out["m_apply"] = apply_bench(B, W, torch, np)

    if not args.no_batched:
        out["multi_system"] = multi_bench(B, W, torch, np, kw)
        out["batched_rhs"] = batched_bench(B, W, torch, np, kw)
        out["powerlaw"] = powerlaw_bench(B, W, torch, np, kw)
        out["gradient"] = gradient_bench(B, W, torch, np)
        out["adaptive_spai"] = adaptive_bench(B, W, torch, np, kw)
        out["bucketed_a"] = bucketed_a_bench(B, W, torch, np, kw)
        out["low_uf_spai"] = low_uf_bench(B, W, torch, np, kw)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.eps, kw)

    # every device object is released before the interpreter exits (a free
    # during interpreter shutdown could run after the HIP runtime's teardown)
    h.free()
    B.release_workspace()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def multi_bench(B, W, torch, np, kw, replays=3):
    """32 uneven 2D variable-coefficient diffusion systems (grid sides 32..448,
    GRF coefficients) in one persistent launch replayed from a captured graph,
    against the same systems solved one gmres_ir_solve after another."""
    c = W.config("4b")
    eps = c["eps"][0]
    systems = []
    for sy in c["systems"]:
        Ad = B.CSRMatrix.from_host(sy["A"])
        h = B.build(Ad, B.CSRMatrix.from_host(sy["P"]), eps=eps, precs=c["precs"])
        systems.append((Ad, torch.as_tensor(sy["b"], device="cuda"), h))
    torch.cuda.synchronize()
    # the largest systems shrink their corrections by less than 2x each under
    # the GMRES cap: no stagnation stop, stop on the residual or on eta
    kw = dict(kw, i_max=64, tol_be=2e-15, stag_ratio=None)
    t0 = time.perf_counter()
    plan = B.MultiPlan(systems, group_blocks=-1, **kw)  # autotuned group size
    tune_s = time.perf_counter() - t0
    plan.launch()
    plan.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        plan.launch()
    sts = plan.wait()
    el = (time.perf_counter() - t0) / replays
    res = {"workload": "32 vardiff2d systems, sides 32..448 (n 4,489..191,844, sum 2,437,223), GRF(16) "
                       "coefficients, buckets fp32/bf16/fp16 eps=1e-2, one persistent launch per replay",
           "systems_per_s": len(systems) / el, "ms_per_replay": el * 1e3, "replays": replays,
           "group_blocks": plan.group_blocks, "autotune_s": tune_s,
           "its_total": [q["its_total"] for q in sts], "max_relres": max(q["relres"][-1] for q in sts),
           "max_eta": max(q["eta"][-1] for q in sts), "stop_reasons": [q["stop_reason"] for q in sts],
           "all_converged": all(q["status"] == 0 for q in sts)}
    plan.free()
    # the same launch with CGS2 orthogonalisation, its group size tuned for it
    t0 = time.perf_counter()
    plan = B.MultiPlan(systems, group_blocks=-1, orth="cgs2", **kw)
    tune2 = time.perf_counter() - t0
    plan.launch()
    plan.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        plan.launch()
    sts = plan.wait()
    el = (time.perf_counter() - t0) / replays
    res["cgs2"] = {"systems_per_s": len(systems) / el, "ms_per_replay": el * 1e3, "group_blocks": plan.group_blocks,
                   "autotune_s": tune2,
                   "its_total": [q["its_total"] for q in sts], "max_relres": max(q["relres"][-1] for q in sts),
                   "all_converged": all(q["status"] == 0 for q in sts)}
    plan.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A, b, h in systems:
        B.solve(A, b, h, **kw)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    res["sequential_systems_per_s"] = len(systems) / seq
    for _, _, h in systems:
        h.free()
    _log(f"multi-system: {res['systems_per_s']:.2f} systems/s (group {res['group_blocks']}), "
         f"CGS2 {res['cgs2']['systems_per_s']:.2f} (group {res['cgs2']['group_blocks']}), sequential {res['sequential_systems_per_s']:.2f}")
    return res


def batched_bench(B, W, torch, np, kw):
    """64 right-hand sides of the 128^3 anisotropic diffusion operator in one
    gmres_ir_solve call (one timed call), against column 0 alone."""
    c = W.config("4a")
    A = c["A"]
    Ad = B.CSRMatrix.from_host(A)
    h = B.build(Ad, B.CSRMatrix.from_host(c["P"]), eps=c["eps"][0], precs=c["precs"])
    Bm = torch.as_tensor(np.ascontiguousarray(c["b"]), device="cuda")
    b0 = Bm[:, 0].contiguous()
    B.solve(Ad, b0, h, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x1, s1 = B.solve(Ad, b0, h, **kw)
    torch.cuda.synchronize()
    single = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, sts = B.solve(Ad, Bm, h, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nr = Bm.shape[1]
    # the MGS passes of the call: a correction runs as many Arnoldi steps as
    # its slowest column; step j makes j + 2 passes over n x R values of u_g:
    # z and v_0 read; z, v_{i-1}, v_i read and z written; z and v_j read and
    # z written
    steps = max(q["steps"] for q in sts)
    per_step = [max(q["its"][i] for q in sts if q["steps"] > i) for i in range(steps)]
    vec = A.n * nr * 4
    mgs_passes = sum(j + 2 for k in per_step for j in range(k))
    mgs_bytes = sum((4 * j + 5) * vec for k in per_step for j in range(k))
    res = {"workload": f"aniso3d 128^3 (1:10:100, n={A.n}), {nr} RHS N(0,1), buckets fp32/bf16/fp16 eps=1e-2",
           "rhs_per_s": nr / el, "s_per_call": el, "single_rhs_per_s": 1.0 / single,
           "arnoldi_steps_per_correction": per_step, "mgs_passes": mgs_passes, "mgs_algorithmic_bytes": mgs_bytes,
           "its_col0": sts[0]["its"], "max_steps": max(q["steps"] for q in sts),
           "max_relres": max(q["relres"][-1] for q in sts), "all_converged": all(q["status"] == 0 for q in sts)}
    del x, Bm
    h.free()
    torch.cuda.empty_cache()
    _log(f"batched: {res['rhs_per_s']:.2f} rhs/s vs single {res['single_rhs_per_s']:.2f}")
    return res


def _converged(st):
    """A solve counts as converged only when it met tol_rr or tol_be."""
    return st["status"] == 0 and st["stop_reason"] in (1, 2)


def _timed_solve(B, torch, Ad, b, h, reps, **kw):
    B.solve(Ad, b, h, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, st = B.solve(Ad, b, h, **kw)
    torch.cuda.synchronize()
    return x, st, (time.perf_counter() - t0) / reps


def _bucket_damage(P, ex, q):
    """Entries that a bucket's format flushed to zero (stored 0, FP64 value not
    0), per bucket, and the zero diagonal entries of M_b."""
    import numpy as np

    lost = (ex["stored"] == 0) & (ex["m64"] != 0)
    flushed = [int(np.count_nonzero(lost & (ex["bucket"] == k))) for k in range(q)]
    rows = np.repeat(np.arange(P.n), np.diff(P.row_ptr))
    zero_diag = int(np.count_nonzero((rows == P.col) & (ex["stored"] == 0)))
    return flushed, zero_diag


def powerlaw_bench(B, W, torch, np, kw, reps=50):
    """The 2^20-row random matrix with power-law rows (mean 13, up to 401,
    lognormal(4) values): SPAI build (rows past the wavefront path go to the
    block path), the bucketed apply with the tuned kernel, and the solve.

    Stopping: the relative residual of this matrix has a floor near 3e-10 of
    ||b|| even with the FP64 M (u |A||x| with entries over 16 orders of
    magnitude), so tol_rr = 1e-10 is unreachable; the solves stop on the
    backward error eta <= 2^-51 (or stagnate).  A solve that meets neither
    test reports no rate.  The eps_b sweep buckets the same FP64 M at each
    eps_b and reports the entries each format flushed to zero, the zero
    diagonal entries of M_b, the iterations and eta, beside the unbucketed
    FP64 M (u_g = fp32) and the all-FP64 SPAI-GMRES-IR."""
    c = W.config("3")
    A, P = c["A"], c["P"]
    n = A.n
    Ad = B.CSRMatrix.from_host(A)
    Pd = B.CSRMatrix.from_host(P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = B.build(Ad, Pd, eps=c["eps"][0], precs=c["precs"])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    h.tune_apply()
    st = h.stats()
    x = torch.randn(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    for _ in range(3):
        B.apply(h, x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.apply(h, x, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nb = sum(1 for cc, p in zip(st["count"], st["precs"]) if cc > 0 and p != 5)
    alg = sum(cc * (VALUE_BYTES[p] + 4) for cc, p in zip(st["count"], st["precs"]) if p != 5)
    alg += 4 * (n + 1) * nb + 8 * n
    ex = h.export()
    h.free()
    del x, y
    b = torch.as_tensor(c["b"], device="cuda")
    kws = dict(kw, tol_rr=0.0, tol_be=2.0 ** -51)
    Md = B.CSRMatrix.from_host(W.CSR(n, P.row_ptr, P.col, ex["m64"]))
    points = []
    for eps in (1e-6, 1e-5, 1e-4, 1e-3):
        he = B.import_m(Md, eps, c["precs"], build_T=False)
        se = he.stats()
        flushed, zdiag = _bucket_damage(P, he.export(), se["q"])
        _, ss, el = _timed_solve(B, torch, Ad, b, he, 3, **kws)
        conv = _converged(ss)
        points.append({"eps": eps, "bucket_counts": se["count"], "flushed_to_zero": flushed, "zero_diagonal": zdiag,
                       "storage_pct": se["storage_pct"], "its": ss["its"], "eta": ss["eta"][-1],
                       "relres": ss["relres"][-1], "status": ss["status"], "stop_reason": ss["stop_reason"],
                       "converged": conv, "solves_per_s": 1.0 / el if conv else None, "s_per_solve": el})
        he.free()
        _log(f"powerlaw eps {eps:g}: counts {se['count']} flushed {flushed} zero diag {zdiag} its {ss['its']} "
             f"eta {ss['eta'][-1]:.2e} relres {ss['relres'][-1]:.2e} stop {ss['stop_reason']}"
             f"{'' if conv else ' (NOT CONVERGED)'}")
    comps = {}
    h64 = B.import_m(Md, 2.0 ** -53, ["fp64"], build_T=False)
    for name, extra in (("spai_fp64M_fp32krylov", {}), ("spai_fp64_all", dict(u_g="fp64", tau=1e-8))):
        _, ss, el = _timed_solve(B, torch, Ad, b, h64, 3, **dict(kws, **extra))
        conv = _converged(ss)
        comps[name] = {"its": ss["its"], "eta": ss["eta"][-1], "relres": ss["relres"][-1], "status": ss["status"],
                       "stop_reason": ss["stop_reason"], "converged": conv,
                       "solves_per_s": 1.0 / el if conv else None}
        _log(f"powerlaw {name}: its {ss['its']} eta {ss['eta'][-1]:.2e} {1.0 / el:.2f} solves/s")
    h64.free()
    del Md
    head = next(p for p in points if p["eps"] == c["eps"][0])
    res = {"workload": f"random n={n}, power-law rows (mean 13, max 401), lognormal(4) values, diagonal 1.1x "
                       f"dominant; SPAI pattern(A), buckets fp64/fp32/fp16/fp8 eps=1e-3; stop on eta <= 2^-51",
           "build_s": build_s, "bucket_counts": st["count"], "storage_pct": st["storage_pct"],
           "apply_kind": st["apply_kind"], "apply_us": ms * 1e3, "apply_algorithmic_bytes": alg,
           "apply_GBs": alg / (ms * 1e-3) / 1e9, "apply_frac_of_peak": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
           "solve_at_eps_1e-3": {k: head[k] for k in ("its", "eta", "relres", "status", "stop_reason", "converged",
                                                      "solves_per_s")},
           "eps_sweep": points, "comparators": comps}
    _log(f"powerlaw: build {build_s:.2f} s, apply {ms * 1e3:.1f} us ({res['apply_GBs']:.0f} GB/s)")
    return res


def gradient_bench(B, W, torch, np):
    """One gradient of L = ||x - x_obs||^2 on the 512^2 variable-coefficient
    system (n = 262,144): forward BSPAI-GMRES-IR, adjoint solve with M_b^T on
    the right, dL/dA_vals; stopping on the backward error with the
    stagnation stop off (see the gradient tests)."""
    c = W.config("5")
    A, P = c["A"], c["P"]
    Ad = B.CSRMatrix.from_host(A)
    h = B.build(Ad, B.CSRMatrix.from_host(P), eps=c["eps"][0], precs=c["precs"])
    kw = dict(tau=1e-4, tol_rr=0.0, tol_be=2e-15, gmres_max=150, i_max=64, stag_ratio=None)
    vals = torch.tensor(A.val, device="cuda", requires_grad=True)
    b = torch.tensor(c["b"], device="cuda", requires_grad=True)
    xobs = torch.zeros(A.n, dtype=torch.float64, device="cuda")

    def step():
        x = B.BSPAISolve.apply(vals, b, Ad, h, kw)
        ((x - xobs) ** 2).sum().backward()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res = {"workload": "vardiff2d 512x512, k = exp(GRF(16)), buckets fp64/fp32/fp16/bf16/fp8 eps=1e-3; forward + "
                       "adjoint GMRES-IR to eta <= 2e-15, gradient in b and A's values",
           "gradients_per_s": 1.0 / el, "s_per_gradient": el, "bucket_counts": h.stats()["count"]}
    h.free()
    _log(f"gradient: {el:.2f} s per forward + adjoint")
    return res


def adaptive_bench(B, W, torch, np, kw, reps=5):
    """The paper's SPAI setting on the 256^2 convection-diffusion system:
    Algorithm 1 with augmentation from an identity start (beta = 8,
    alpha = 5, eps = 0.4), bucketed as the headline (eps_b = 1e-4,
    fp64/fp32/fp16/bf16), against the fixed pattern(A^2) SPAI."""
    c = W.config("2")
    A, P = c["A"], c["P"]
    Ad = B.CSRMatrix.from_host(A)
    b = torch.as_tensor(c["b"], device="cuda")
    res = {"workload": "convdiff2d 256x256 (n=65536); adaptive SPAI from the identity, alpha=5 beta=8 eps=0.4; "
                       "buckets fp64/fp32/fp16/bf16 eps_b=1e-4"}
    for name, make in (("adaptive", lambda: B.build_adaptive(Ad, alpha=5, beta=8, eps_spai=0.4, precs=c["precs"],
                                                             eps=1e-4)),
                       ("pattern_A2", lambda: (B.build(Ad, B.CSRMatrix.from_host(P), eps=1e-4, precs=c["precs"]),
                                               None))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, steps = make()
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        st = h.stats()
        B.solve(Ad, b, h, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, ss = B.solve(Ad, b, h, **kw)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        res[name] = {"build_s": build_s, "nnz_M": int(sum(st["count"])), "bucket_counts": st["count"],
                     "storage_pct": st["storage_pct"], "its": ss["its"], "relres": ss["relres"][-1],
                     "solves_per_s": 1.0 / el}
        if steps is not None:
            res[name]["solves_per_row_histogram"] = np.bincount(steps).tolist()
        h.free()
        _log(f"{name}: build {build_s * 1e3:.1f} ms, nnz(M) {res[name]['nnz_M']}, its {ss['its']}, "
             f"{1.0 / el:.2f} solves/s")
    return res


def bucketed_a_bench(B, W, torch, np, kw, reps=5):
    """A bucketed inside GMRES too (eqs. (nbe2), (fe2)) on the 256^2
    convection-diffusion system, M as the headline (eps_b = 1e-4): per eps of
    A, its bucket counts, the bytes of one product with A_b, iterations,
    backward error and solve rate, against A rounded to fp32."""
    c = W.config("2")
    A, P = c["A"], c["P"]
    Ad = B.CSRMatrix.from_host(A)
    b = torch.as_tensor(c["b"], device="cuda")
    h = B.build(Ad, B.CSRMatrix.from_host(P), eps=1e-4, precs=c["precs"])
    res = {"workload": "convdiff2d 256x256 (n=65536), M pattern(A^2) eps_b=1e-4; A bucketed fp64/fp32/fp16/bf16 "
                       "at eps_A", "points": []}
    vbytes = {0: 8, 1: 4, 2: 2, 3: 2, 4: 1}

    def run(hA):
        B.solve(Ad, b, h, A_b=hA, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, ss = B.solve(Ad, b, h, A_b=hA, **kw)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        return ss, el

    ss, el = run(None)
    res["plain_fp32"] = {"a_value_bytes": 4 * A.nnz, "its": ss["its"], "its_total": ss["its_total"],
                         "relres": ss["relres"][-1], "eta": ss["eta"][-1], "solves_per_s": 1.0 / el}
    _log(f"A rounded to fp32: its {ss['its']} {1.0 / el:.2f} solves/s")
    for eps in (1e-6, 1e-4, 1e-2):
        hA = B.bucket_a(Ad, eps, c["precs"])
        st = hA.stats()
        ss, el = run(hA)
        vb = int(sum(cnt * vbytes[p] for cnt, p in zip(st["count"], [0, 1, 2, 3])))
        res["points"].append({"eps_A": eps, "bucket_counts": st["count"], "a_value_bytes": vb, "its": ss["its"],
                              "its_total": ss["its_total"], "relres": ss["relres"][-1], "eta": ss["eta"][-1],
                              "stop_reason": ss["stop_reason"], "solves_per_s": 1.0 / el})
        _log(f"A_b eps {eps:g}: counts {st['count']} its {ss['its']} eta {ss['eta'][-1]:.2e} "
             f"{1.0 / el:.2f} solves/s")
        hA.free()
    h.free()
    return res


def low_uf_bench(B, W, torch, np, kw, reps=5):
    """The SPAI least squares in u_f = fp64, fp32 and fp16 (Section 4's
    settings, with its column scaling) on the 256^2 convection-diffusion
    system, pattern(A^2), bucketed at eps_b = 1e-4: build time (median of 5),
    the bucket counts, iterations and solve rate of the resulting M."""
    c = W.config("2")
    A, P = c["A"], c["P"]
    Ad = B.CSRMatrix.from_host(A)
    Pd = B.CSRMatrix.from_host(P)
    b = torch.as_tensor(c["b"], device="cuda")
    res = {"workload": "convdiff2d 256x256 (n=65536), SPAI pattern(A^2) with column scaling, buckets "
                       "fp64/fp32/fp16/bf16 eps_b=1e-4"}
    for uf in ("fp64", "fp32", "fp16"):
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = B.build(Ad, Pd, eps=1e-4, precs=c["precs"], scale=True, u_f=uf)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            st = h.stats()
            if len(times) < 5:
                h.free()
        B.solve(Ad, b, h, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, ss = B.solve(Ad, b, h, **kw)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        res[uf] = {"build_ms": 1e3 * float(np.median(times)), "bucket_counts": st["count"],
                   "storage_pct": st["storage_pct"], "its": ss["its"], "relres": ss["relres"][-1],
                   "eta": ss["eta"][-1], "solves_per_s": 1.0 / el}
        h.free()
        _log(f"u_f {uf}: build {res[uf]['build_ms']:.2f} ms, counts {st['count']}, its {ss['its']}, "
             f"{1.0 / el:.2f} solves/s")
    return res


def apply_bench(B, W, torch, np):
    """bspai_apply on the 128^3 anisotropic operator (n = 2,097,152, M on the
    pattern of A, all entries in the bf16 bucket at eps = 1e-2), cold in HBM:
    the product rotates over 8 copies of M and of x/y (about 0.9 GB)."""
    _log("apply bench: building 128^3 operator")
    c = W.config("4a")
    A = c["A"]
    Ad = B.CSRMatrix.from_host(A)
    h0 = B.build(Ad, B.CSRMatrix.from_host(c["P"]), eps=1e-2, precs=c["precs"], build_T=False, keep_fp64_M=True)
    ex = h0.export()
    h0.free()
    M = W.CSR(A.n, c["P"].row_ptr, c["P"].col, ex["m64"])
    Md = B.CSRMatrix.from_host(M)
    copies = 8
    hs = [B.import_m(Md, 1e-2, c["precs"], build_T=False, keep_fp64_M=False) for _ in range(copies)]
    st = hs[0].stats()
    n = A.n
    xs = [torch.randn(n, device="cuda", dtype=torch.float32) for _ in range(copies)]
    ys = [torch.empty(n, device="cuda", dtype=torch.float32) for _ in range(copies)]
    nb = sum(1 for cc, p in zip(st["count"], st["precs"]) if cc > 0 and p != 5)
    bytes_per = sum(cc * (VALUE_BYTES[p] + 4) for cc, p in zip(st["count"], st["precs"]) if p != 5)
    bytes_per += 4 * (n + 1) * nb + 4 * n + 4 * n
    # bytes the product copies actually hold: ELL copies n W (value + column
    # code) bytes, other buckets their CSR bytes
    moved = 8 * n
    for cc, p, w, cb in zip(st["count"], st["precs"], st["ell_width"], st["col_bytes"]):
        if p == 5 or cc == 0:
            continue
        moved += n * w * (VALUE_BYTES[p] + cb) if w else cc * (VALUE_BYTES[p] + 4) + 4 * (n + 1)
    for i in range(copies):
        B.apply(hs[i], xs[i], ys[i])
    torch.cuda.synchronize()
    reps = int(os.environ.get("BSPAI_APPLY_REPS", "200"))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # launches captured in a graph: the replay times the kernels, not the
    # Python-side call overhead of each apply
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        for i in range(copies):
            B.apply(hs[i], xs[i], ys[i])
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for r in range(reps):
            B.apply(hs[r % copies], xs[r % copies], ys[r % copies])
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # the same launches issued one by one from Python, for reference
    e0.record()
    for r in range(reps):
        B.apply(hs[r % copies], xs[r % copies], ys[r % copies])
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / reps
    for hh in hs:
        hh.free()
    gbs = bytes_per / (ms * 1e-3) / 1e9
    _log(f"apply: {ms * 1e3:.1f} us per launch, {gbs:.0f} GB/s (issued from Python one by one: {ms_eager * 1e3:.1f} us)")
    return {"workload": "aniso3d 128^3 7-point (n=2097152), M on pattern(A), bf16 bucket (eps=1e-2), fp32 x/y, "
                        "8 rotating copies (cold HBM), launches replayed from a captured graph", "bucket_counts": st["count"],
            "us_per_launch": ms * 1e3, "us_per_launch_python_issued": ms_eager * 1e3,
            "algorithmic_bytes": bytes_per, "achieved_GBs": gbs, "frac_of_peak": gbs / PEAK_HBM_GBS,
            "bytes_per_nnz": bytes_per / max(1, sum(st["count"])), "ell_width": st["ell_width"],
            "col_bytes": st["col_bytes"], "moved_bytes": moved, "moved_GBs": moved / (ms * 1e-3) / 1e9,
            "traffic": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "apply.hip"),
                                "apply_kernel_traffic.json")}


def cpu_baseline(c, eps, kw):
    """The CPU oracle (plain C, OpenMP over rows, sequential dot products
    accumulated in FP64, the realisation the GPU computes) on the same
    workload: one full solve from the FP64 SPAI (SPAI build not timed)."""
    import oracle as O
    import workloads as W

    A, P = c["A"], c["P"]
    threads = O.num_threads(0)
    st, Mv, _ = O.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    Mb = O.Bucketed(M, eps, c["precs"])
    t0 = time.perf_counter()
    res = O.gmres_ir(A, M, Mb, c["b"], dot64=True, **kw)
    el = time.perf_counter() - t0
    _log(f"oracle: {el:.1f} s per solve on {threads} threads, its {res['its']}")
    return {"value": 1.0 / el, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one full solve of the same workload (its {res['its']}, {el:.1f} s)",
            "eta": res["eta"][-1]}


if __name__ == "__main__":
    main()
