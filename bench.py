#!/usr/bin/env python
"""BSPAI-GMRES-IR on one MI355X: right-hand-side solves/s and bucketed M-apply
bandwidth, BSPAI against all-FP64 SPAI at equal stopping tests.

Headline workload: the 128^3 anisotropic 7-point diffusion operator
(1:10:100, n = 2,097,152) with 64 right-hand sides N(0,1) sharing one BSPAI
M (SPAI on the pattern of A, buckets fp32/fp16/bf16 at eps_b = 1e-2),
u_g = u_p = fp32, u = fp64, residuals in double-double, tau = 1e-4, refinement
to relative residual 1e-10, GMRES cap 50 (each correction's Arnoldi run
stops at 50 steps; the solve takes about a dozen corrections).  The library
solves many
right-hand sides in column groups (4 columns in FP32, one cooperative MGS
launch per Arnoldi step); a step is one gmres_ir_solve call on one such group
of 4 of the 64 columns, the steps cycling through the 16 groups.  value =
right-hand sides solved per second.  A, M and b are resident on the GPU
before timing starts.

Printed (one JSON line): the headline with the MGS kernel's roofline
(algorithmic bytes / kernel time, HIP events recorded by the library on the
solve's stream), the all-FP64 SPAI-GMRES-IR comparator at the same stopping
test, the CPU oracle timed on the host, and secondary blocks (the 256^2
convection-diffusion solve and its latency floor, the cold bucketed apply,
the 32-system launch, the power-law matrix, the gradient, adaptive SPAI,
bucketed A, low-u_f SPAI).
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
GROUP = 4  # columns per step: the library's FP32 column group (16 bytes of u_g per row)


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


def _traffic(kernel_src, record="solve_kernel_traffic.json", alg_bytes=None):
    """HBM traffic per launch from the committed rocprofv3 counter runs, only if
    they were taken on the current kernel source (and, given alg_bytes, on a
    workload of the same algorithmic bytes per launch, within 1%)."""
    p = os.path.join(ROOT, "profiles", record)
    try:
        with open(p) as f:
            t = json.load(f)
        if t.get("source_sha256_16") != _src_hash(kernel_src):
            return None
        ref = t.get("algorithmic_bytes_per_launch")
        if alg_bytes is not None and (not ref or abs(ref / alg_bytes - 1.0) > 0.01):
            return None
        return t.get("bytes_per_launch")
    except (OSError, ValueError, ZeroDivisionError):
        pass
    return None


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


def _cols_summary(sts):
    return {"its_col0": sts[0]["its"], "max_steps": max(q["steps"] for q in sts),
            "max_relres": max(q["relres"][-1] for q in sts), "max_eta": max(q["eta"][-1] for q in sts),
            "all_converged": all(_converged(q) for q in sts)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--gmres-max", type=int, default=150, help="GMRES cap of the secondary workloads")
    ap.add_argument("--headline-cap", type=int, default=50,
                    help="GMRES cap of the headline solve (its MGS work per correction grows as the cap squared)")
    ap.add_argument("--i-max", type=int, default=20, help="refinement corrections allowed per solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="only the headline (and its comparators)")
    ap.add_argument("--no-comparators", action="store_true",
                    help="the headline's timed steps only (no one-call and FP64 comparator runs): profiling")
    ap.add_argument("--only-apply", action="store_true", help="run only the cold bucketed-apply measurement")
    ap.add_argument("--only-convdiff", action="store_true", help="run only the 256^2 convection-diffusion block")
    ap.add_argument("--only-multi", action="store_true", help="run only the 32-system measurement")
    ap.add_argument("--only-powerlaw", action="store_true", help="run only the power-law matrix measurement")
    ap.add_argument("--only-powerlaw-apply", action="store_true",
                    help="run only the power-law matrix's build and apply timings (no solves)")
    ap.add_argument("--only-gradient", action="store_true", help="run only the 512^2 gradient measurement")
    ap.add_argument("--only-adaptive", action="store_true", help="run only the adaptive-SPAI measurement")
    ap.add_argument("--only-bucketed-a", action="store_true", help="run only the bucketed-A measurement")
    ap.add_argument("--only-low-uf", action="store_true", help="run only the low-u_f SPAI measurement")
    ap.add_argument("--only-cpu-baseline", action="store_true", help="run only the oracle on the host")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy first (calibration of hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only (every kernel works on one GPU's memory); "
                                   "run with --gpus 1"}), flush=True)
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
    kw0 = dict(tau=1e-4, tol_rr=1e-10, gmres_max=args.gmres_max, i_max=args.i_max)
    kwh = dict(kw0, gmres_max=args.headline_cap)
    if args.only_apply:
        _emit(B, torch, {"m_apply": apply_bench(B, W, torch, np)})
        return
    if args.only_convdiff:
        _emit(B, torch, {"convdiff_256": convdiff_bench(B, W, torch, np, kw0, args.steps, args.warmup)})
        return
    if args.only_multi:
        _emit(B, torch, {"multi_system": multi_bench(B, W, torch, np, kw0)})
        return
    if args.only_powerlaw:
        _emit(B, torch, {"powerlaw": powerlaw_bench(B, W, torch, np, kw0)})
        return
    if args.only_powerlaw_apply:
        _emit(B, torch, {"powerlaw": powerlaw_bench(B, W, torch, np, kw0, reps=20, apply_only=True)})
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
    if args.only_cpu_baseline:
        _emit(B, torch, {"cpu_baseline": cpu_baseline(W, np, kwh, [args.headline_cap] * 12)})
        return

    out, its_per_col = headline(B, W, torch, np, kwh, args.steps, args.warmup, not args.no_comparators)
    if not args.no_secondary:
        out["convdiff_256"] = convdiff_bench(B, W, torch, np, kw0, 20, 3)
        out["m_apply"] = apply_bench(B, W, torch, np)
        out["multi_system"] = multi_bench(B, W, torch, np, kw0)
        out["powerlaw"] = powerlaw_bench(B, W, torch, np, kw0)
        out["gradient"] = gradient_bench(B, W, torch, np)
        out["adaptive_spai"] = adaptive_bench(B, W, torch, np, kw0)
        out["bucketed_a"] = bucketed_a_bench(B, W, torch, np, kw0)
        out["low_uf_spai"] = low_uf_bench(B, W, torch, np, kw0)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, np, kwh, its_per_col)
    _emit(B, torch, out)


def headline(B, W, torch, np, kw, steps, warmup, comparators=True):
    """The 64-RHS 128^3 workload: K timed steps of one 4-column group each
    (cycling over the 16 groups), the MGS kernel's roofline, and the all-FP64
    SPAI-GMRES-IR comparator at the same stopping test."""
    _log("headline: generating the 128^3 operator and 64 right-hand sides")
    c = W.config("4a")
    A, P = c["A"], c["P"]
    n = A.n
    Ad = B.CSRMatrix.from_host(A)
    Pd = B.CSRMatrix.from_host(P)
    Bm = torch.as_tensor(np.ascontiguousarray(c["b"]), device="cuda")
    nr = Bm.shape[1]
    groups = [Bm[:, k:k + GROUP].contiguous() for k in range(0, nr, GROUP)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = B.build(Ad, Pd, eps=c["eps"][0], precs=c["precs"])
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    mst = h.stats()
    _log(f"built M: counts {mst['count']} storage {mst['storage_pct']:.1f}% in {build_s * 1e3:.0f} ms")
    for w in range(warmup):
        B.solve(Ad, groups[w % len(groups)], h, **kw)
    torch.cuda.synchronize()
    B.set_profiling(True)
    B.batched_mgs_profile(reset=True)
    sts_all = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        _, sts = B.solve(Ad, groups[k % len(groups)], h, **kw)
        sts_all.extend(sts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.set_profiling(False)
    prof = B.batched_mgs_profile(reset=True)
    rhs_per_s = GROUP * steps / elapsed
    summ = _cols_summary(sts_all)
    _log(f"BSPAI: {rhs_per_s:.2f} RHS/s ({elapsed * 1e3 / steps:.0f} ms per {GROUP}-column step), "
         f"its {summ['its_col0']}, max relres {summ['max_relres']:.2e}, all converged {summ['all_converged']}")
    mgs_gbs = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] > 0 else 0.0
    alg_launch = prof["bytes"] / max(1, prof["launches"])
    avg_us = 1e3 * prof["ms"] / max(1, prof["launches"])
    roofline = {"kernel": "k_b_mgs_persist (one Arnoldi step's MGS for a 4-column group)", "bound": "hbm",
                "achieved": mgs_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": mgs_gbs / PEAK_HBM_GBS,
                "traffic": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "solve.hip"),
                                    "batched_mgs_traffic.json", alg_launch),
                "launches": prof["all_launches"], "launches_timed": prof["launches"],
                "timing": "HIP events around one launch in seven (the count runs over every j)",
                "avg_launch_us": avg_us, "algorithmic_bytes_per_launch": alg_launch,
                "kernel_share_of_step": avg_us * 1e-6 * prof["all_launches"] / elapsed}
    out = {"metric": "GMRES-IR solves/s & M-apply HBM GB/s, BSPAI vs fp64 SPAI at equal backward error",
           "value": rhs_per_s, "unit": "RHS solves/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"aniso3d 128^3 7-point 1:10:100 (n={n}), {nr} RHS N(0,1) sharing one BSPAI M "
                                  f"(SPAI pattern(A) FP64, buckets fp32/fp16/bf16 eps=1e-2), u_g=u_p=fp32, "
                                  f"u_r=double-double, tau=1e-4, refine to 1e-10 rel. residual, GMRES cap "
                                  f"{kw['gmres_max']}; a step solves one {GROUP}-column group, cycling over the "
                                  f"{nr // GROUP} groups",
                      "n": n, "nnz_A": A.nnz, "nnz_M": int(sum(mst["count"])), "bucket_counts": mst["count"],
                      "storage_pct": mst["storage_pct"], "rhs": nr, "columns_per_step": GROUP},
           "solve": dict(summ, build_ms=build_s * 1e3),
           "roofline": roofline}

    if not comparators:
        h.free()
        return out, sts_all[0]["its"]
    # the same 64 columns in one call (the library runs its 16 groups)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sts = B.solve(Ad, Bm, h, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["one_call_64_rhs"] = dict(_cols_summary(sts), s_per_call=el, rhs_per_s=nr / el)
    _log(f"one call, 64 RHS: {el:.2f} s ({nr / el:.2f} RHS/s)")

    # comparators at the same stopping test: the all-FP64 SPAI-GMRES-IR (one
    # fp64 bucket, u_g = u_p = fp64, tau = 1e-8) and the FP64 M with the FP32
    # Krylov solve (isolates the bucketing)
    ex = h.export()
    Md = B.CSRMatrix.from_host(W.CSR(n, P.row_ptr, P.col, ex["m64"]))
    h64 = B.import_m(Md, 2.0 ** -53, ["fp64"], build_T=False)
    del Md, ex
    comps = {}
    for name, extra, reps in (("spai_fp64_all", dict(u_g="fp64", tau=1e-8), 3),
                              ("spai_fp64M_fp32krylov", {}, 3)):
        k2 = dict(kw, **extra)
        B.solve(Ad, groups[0], h64, **k2)
        torch.cuda.synchronize()
        sts_c = []
        t0 = time.perf_counter()
        for k in range(reps):
            _, sts = B.solve(Ad, groups[k % len(groups)], h64, **k2)
            sts_c.extend(sts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        comps[name] = dict(_cols_summary(sts_c), rhs_per_s=GROUP * reps / el, rhs_timed=GROUP * reps)
        _log(f"{name}: {GROUP * reps / el:.2f} RHS/s, its {sts_c[0]['its']}, max eta {comps[name]['max_eta']:.2e}")
    h64.free()
    out["comparators"] = comps
    out["speedup_vs_fp64_spai"] = rhs_per_s / comps["spai_fp64_all"]["rhs_per_s"]
    h.free()
    del groups, Bm
    torch.cuda.empty_cache()
    its_per_col = sts_all[0]["its"]
    return out, its_per_col


def convdiff_bench(B, W, torch, np, kw, steps, warmup):
    """The 256 x 256 upwind convection-diffusion system (n = 65,536, Peclet
    50), SPAI on the pattern of A^2 in FP64, buckets {fp64, fp32, fp16, bf16}
    at eps_b = 1e-4, b = A x_true: solves/s of the persistent single-system
    solver, its roofline and latency floor, comparators and the eps_b sweep."""
    c = W.config("2")
    A, P = c["A"], c["P"]
    n = A.n
    Ad = B.CSRMatrix.from_host(A)
    Pd = B.CSRMatrix.from_host(P)
    b = torch.as_tensor(c["b"], device="cuda")
    precs = c["precs"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = B.build(Ad, Pd, eps=1e-4, precs=precs)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    mst = h.stats()
    for _ in range(warmup):
        x, st = B.solve(Ad, b, h, **kw)
    torch.cuda.synchronize()
    B.set_profiling(True)
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        x, stats = B.solve(Ad, b, h, **kw)
        kernel_ms.append(B.last_solve_kernel_ms())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.set_profiling(False)
    solves_per_s = steps / elapsed
    xh = x.cpu().numpy()
    fwd = float(np.abs(xh - c["x_true"]).max() / np.abs(c["x_true"]).max())
    _log(f"convdiff 256^2: {solves_per_s:.2f} solves/s, its {stats['its']}, relres {stats['relres'][-1]:.2e}")
    kern_ms = float(np.mean(kernel_ms))
    nbytes = solve_bytes(stats, n, A.nnz, mst)
    G = B.solve_blocks(n)
    ex_us = B.exchange_latency_us(G)
    n_ex = 3 + sum(6 + sum(j + 4 for j in range(k)) for k in stats["its"])
    res = {"workload": "convdiff2d 256x256 upwind Pe=50 (n=65536), SPAI pattern(A^2) FP64, buckets "
                       "fp64/fp32/fp16/bf16 eps=1e-4, u_g=u_p=fp32, u_r=double-double, tau=1e-4, refine to 1e-10",
           "solves_per_s": solves_per_s, "ms_per_solve": elapsed * 1e3 / steps, "steps": steps,
           "bucket_counts": mst["count"], "storage_pct": mst["storage_pct"], "its": stats["its"],
           "relres": stats["relres"][-1], "eta": stats["eta"][-1], "forward_error": fwd,
           "converged": _converged(stats), "build_ms": build_ms,
           "roofline": {"kernel": "k_gmres_ir (persistent solver)", "bound": "hbm",
                        "achieved": nbytes / (kern_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": nbytes / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                        "traffic": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "solve.hip")),
                        "algorithmic_bytes": nbytes, "kernel_ms": kern_ms},
           "latency_floor": {"blocks": G, "exchange_us": ex_us, "exchanges_per_solve": n_ex,
                             "floor_ms": n_ex * ex_us * 1e-3, "frac": n_ex * ex_us * 1e-3 / kern_ms}}
    _log(f"latency floor: {n_ex} exchanges x {ex_us:.2f} us = {n_ex * ex_us * 1e-3:.1f} ms "
         f"({100 * n_ex * ex_us * 1e-3 / kern_ms:.0f}% of the kernel time)")
    # the exchange with the blocks on one XCD against the dispatcher's spread
    place = {}
    for G2 in (16, 32):
        one, xo = B.exchange_latency_placed_us(G2, True)
        spread, _ = B.exchange_latency_placed_us(G2, False)
        place[str(G2)] = {"one_xcd_us": one, "spread_us": spread, "xcds_one": sorted(set(xo))}
    res["exchange_placement"] = place
    comps = {}
    h64 = B.build(Ad, Pd, eps=2.0 ** -53, precs=["fp64"])
    for name, hh, extra in (("spai_fp64_all", h64, dict(u_g="fp64", tau=1e-8)),
                            ("spai_fp64M_fp32krylov", h64, {}),
                            ("bspai_cgs2", h, dict(orth="cgs2"))):
        _, s2, el = _timed_solve(B, torch, Ad, b, hh, 5, **dict(kw, **extra))
        comps[name] = {"solves_per_s": 1.0 / el, "its": s2["its"], "relres": s2["relres"][-1], "eta": s2["eta"][-1],
                       "converged": _converged(s2)}
        _log(f"{name}: {1.0 / el:.2f} solves/s its {s2['its']}")
    h64.free()
    res["comparators"] = comps
    sweep = []
    for eps in (1e-6, 1e-4, 1e-2):
        he = B.build(Ad, Pd, eps=eps, precs=precs)
        se = he.stats()
        _, ste, el = _timed_solve(B, torch, Ad, b, he, 3, **kw)
        sweep.append({"eps": eps, "bucket_counts": se["count"], "storage_pct": se["storage_pct"], "its": ste["its"],
                      "its_total": ste["its_total"], "eta": ste["eta"][-1], "relres": ste["relres"][-1],
                      "converged": _converged(ste), "solves_per_s": 1.0 / el})
        he.free()
    res["eps_sweep"] = {"plain_spai_its": comps["spai_fp64M_fp32krylov"]["its"], "points": sweep}
    h.free()
    return res


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


def _bucket_damage(P, ex, q):
    """Entries that a bucket's format flushed to zero (stored 0, FP64 value not
    0), per bucket, and the zero diagonal entries of M_b."""
    import numpy as np

    lost = (ex["stored"] == 0) & (ex["m64"] != 0)
    flushed = [int(np.count_nonzero(lost & (ex["bucket"] == k))) for k in range(q)]
    rows = np.repeat(np.arange(P.n), np.diff(P.row_ptr))
    zero_diag = int(np.count_nonzero((rows == P.col) & (ex["stored"] == 0)))
    return flushed, zero_diag


def powerlaw_bench(B, W, torch, np, kw, reps=50, apply_only=False):
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
    x = torch.randn(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)

    def time_apply():
        for _ in range(3):
            B.apply(h, x, out=y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            B.apply(h, x, out=y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    by_kind = {}
    for kind, name in ((2, "lds_tiles"), (4, "lanes_per_row"), (5, "entry_balanced_tiles")):
        try:
            h.set_apply_kind(kind)
        except B.BSPAIError:
            continue
        by_kind[name] = time_apply() * 1e3
    h.tune_apply()
    st = h.stats()
    ms = time_apply()
    nb = sum(1 for cc, p in zip(st["count"], st["precs"]) if cc > 0 and p != 5)
    alg = sum(cc * (VALUE_BYTES[p] + 4) for cc, p in zip(st["count"], st["precs"]) if p != 5)
    alg += 4 * (n + 1) * nb + 8 * n
    if apply_only:
        h.free()
        return {"workload": "random n=%d, power-law rows, SPAI pattern(A), buckets eps=1e-3" % n,
                "bucket_counts": st["count"], "apply_kind": st["apply_kind"], "apply_us": ms * 1e3,
                "apply_us_by_kernel": by_kind, "apply_algorithmic_bytes": alg,
                "apply_GBs": alg / (ms * 1e-3) / 1e9,
                "traffic_bytes_per_launch": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "apply.hip"),
                                                     "powerlaw_apply_traffic.json")}
    ex = h.export()
    h.free()
    del x, y
    b = torch.as_tensor(c["b"], device="cuda")
    kws = dict(kw, tol_rr=0.0, tol_be=2.0 ** -51)
    Md = B.CSRMatrix.from_host(W.CSR(n, P.row_ptr, P.col, ex["m64"]))
    points = []
    for eps in (1e-9, 1e-8, 1e-7, 1e-6, 1e-5, 1e-3):
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
           "apply_kind": st["apply_kind"], "apply_us": ms * 1e3, "apply_us_by_kernel": by_kind,
           "apply_algorithmic_bytes": alg,
           "apply_traffic_bytes_per_launch": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "apply.hip"),
                                                      "powerlaw_apply_traffic.json"),
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


def _apply_cold(B, torch, Md, precs, eps, n, copies=8):
    """Cold bspai_apply: the product rotates over `copies` independently
    bucketed copies of M and of x/y (more than the 256 MiB Infinity Cache),
    launches replayed from a captured graph."""
    hs = [B.import_m(Md, eps, precs, build_T=False, keep_fp64_M=False) for _ in range(copies)]
    st = hs[0].stats()
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
    del graph
    for hh in hs:
        hh.free()
    gbs = bytes_per / (ms * 1e-3) / 1e9
    _log(f"apply eps {eps:g}: counts {st['count']}, {ms * 1e3:.1f} us per launch, {gbs:.0f} GB/s algorithmic, "
         f"{moved / (ms * 1e-3) / 1e9:.0f} GB/s of stored bytes")
    return {"eps": eps, "bucket_counts": st["count"], "us_per_launch": ms * 1e3, "algorithmic_bytes": bytes_per,
            "achieved_GBs": gbs, "frac_of_peak": gbs / PEAK_HBM_GBS,
            "bytes_per_nnz": bytes_per / max(1, sum(st["count"])), "ell_width": st["ell_width"],
            "col_bytes": st["col_bytes"], "apply_kind": st["apply_kind"], "moved_bytes": moved,
            "moved_GBs": moved / (ms * 1e-3) / 1e9, "moved_frac_of_peak": moved / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}


def apply_bench(B, W, torch, np):
    """bspai_apply on the 128^3 anisotropic operator (n = 2,097,152, M on the
    pattern of A), cold in HBM: at eps_b = 1e-2 (every entry in the bf16
    bucket) and at 1e-4 (fp32, fp16 and bf16 buckets all non-empty).  Two
    rates: algorithmic bytes (an int32 column per entry) and the bytes the
    product's copies actually hold (1-byte column codes where they apply);
    the counters' HBM traffic is recorded for the single-bucket case."""
    _log("apply bench: building 128^3 operator")
    c = W.config("4a")
    A = c["A"]
    Ad = B.CSRMatrix.from_host(A)
    h0 = B.build(Ad, B.CSRMatrix.from_host(c["P"]), eps=1e-2, precs=c["precs"], build_T=False, keep_fp64_M=True)
    ex = h0.export()
    h0.free()
    Md = B.CSRMatrix.from_host(W.CSR(A.n, c["P"].row_ptr, c["P"].col, ex["m64"]))
    res = {"workload": "aniso3d 128^3 7-point (n=2097152), M on pattern(A), buckets fp32/fp16/bf16, fp32 x/y, "
                       "8 rotating copies (cold HBM), launches replayed from a captured graph",
           "points": [_apply_cold(B, torch, Md, c["precs"], eps, A.n) for eps in (1e-2, 1e-4)],
           "traffic_eps_1e-2": _traffic(os.path.join(ROOT, "paper_2307_03914_amd", "csrc", "apply.hip"),
                                        "apply_kernel_traffic.json")}
    del Md
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, np, kw, its_per_col):
    """The CPU oracle (plain C, OpenMP over rows, dot products sequential and
    accumulated in FP64, the realisation the GPU computes) on the headline
    workload, one column.  A full solve of one column is about a dozen
    corrections of 50 GMRES iterations (minutes on the host), so the sample
    is bounded:
    MGS-GMRES corrections of 20 and 40 iterations on M_b A d = M_b r fix
    t(k) = a k + b k (k + 1) / 2 (the products per iteration, the
    Gram-Schmidt growing with k), which is summed over the column's GPU
    iteration counts.  The 1-thread figure fits corrections of 10 and 20
    iterations at 1 thread.  Also the oracle's bucketed apply on the same M."""
    import oracle as O

    c = W.config("4a")
    A, P = c["A"], c["P"]
    threads = O.num_threads(0)
    st, Mv, _ = O.spai(A, P)
    M = W.CSR(A.n, P.row_ptr, P.col, Mv)
    Mb = O.Bucketed(M, c["eps"][0], c["precs"])
    r = np.ascontiguousarray(c["b"][:, 0])
    # the oracle's M-apply rate (FP64-mode product of the stored values)
    x = np.random.default_rng(0).standard_normal(A.n)
    O.apply(Mb, x)
    t0 = time.perf_counter()
    for _ in range(3):
        O.apply(Mb, x)
    t_apply = (time.perf_counter() - t0) / 3
    nb = sum(1 for cc in Mb.counts if cc > 0)
    alg = sum(int(cc) * (VALUE_BYTES[p] + 4) for cc, p in zip(Mb.counts, Mb.precs)) + 4 * (A.n + 1) * nb + 8 * A.n

    def timed(k):
        t0 = time.perf_counter()
        g = O.gmres(A, Mb, r, tau=0.0, max_it=k, dot64=True)
        assert g["its"] == k, g["its"]
        return time.perf_counter() - t0

    def per_rhs(k1, k2):
        t1, t2 = timed(k1), timed(k2)
        q = lambda k: k * (k + 1) / 2.0
        det = k1 * q(k2) - k2 * q(k1)
        a = (t1 * q(k2) - t2 * q(k1)) / det
        b = (k1 * t2 - k2 * t1) / det
        return sum(a * k + b * q(k) for k in its_per_col), (t1, t2)

    sec, (t20, t40) = per_rhs(20, 40)
    O.num_threads(1)
    sec1, (t10_1, t20_1) = per_rhs(10, 20)
    O.num_threads(threads)
    _log(f"oracle: 20/40 iterations {t20:.1f}/{t40:.1f} s on {threads} threads -> {sec:.0f} s per RHS; 1 thread "
         f"10/20 iterations {t10_1:.1f}/{t20_1:.1f} s -> {sec1:.0f} s per RHS; apply {t_apply * 1e3:.0f} ms")
    return {"value": 1.0 / sec, "unit": "RHS solves/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"one column of the 128^3 64-RHS workload: GMRES corrections of 20 and 40 iterations "
                      f"({t20:.1f} s, {t40:.1f} s on {threads} threads) fitting t(k) = a k + b k(k+1)/2, summed "
                      f"over the column's GPU iteration counts {its_per_col}",
            "value_1_thread": 1.0 / sec1,
            "sample_1_thread": f"corrections of 10 and 20 iterations on 1 thread ({t10_1:.1f} s, {t20_1:.1f} s), "
                               f"the same fit",
            "apply_GBs": alg / t_apply / 1e9, "apply_ms": t_apply * 1e3}


if __name__ == "__main__":
    main()
