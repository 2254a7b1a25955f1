#!/usr/bin/env python3
"""Benchmark: TV/L2 reconstructions per second on one MI355X.

Workload (the single-image configuration of the method's dense-A path): n = 128
(16384 pixels), m = 4096 Gaussian rows (25 %), FP32 A (256 MiB), 20 random
rectangles/disks plus a linear ramp, noise sigma = 1e-3, mu = 1e3, beta = 10,
500 iterations of the accelerated inexact ADM (Alg. 2), tol = 0.  One step is
one full reconstruction; inputs are resident in HBM before the timed region.

Prints one JSON line with the throughput, the roofline of the dominant kernel
(the one-pass product g = A^T (A u - f), timed with HIP events on the stream it
runs on), the FP64
oracle timed on the host cores, and the relative error of the GPU result
against that oracle run (same tau on both sides).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_gemv_n128_m4096.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary of the n = 128, m = 4096 products (None if absent)."""
    try:
        for line in open(TRAFFIC_FILE):
            if line.startswith(f"traffic_bytes_per_launch {kernel}:"):
                return float(line.split(":")[1])
    except OSError:
        pass
    return None


def psnr_db(u, ref):
    """PSNR of u against the FP64 reference: 20 log10(max |ref| / RMS(u - ref))."""
    import numpy as np
    rms = float(np.sqrt(np.mean((np.asarray(u, np.float64) - ref) ** 2)))
    return float("inf") if rms == 0.0 else float(20.0 * np.log10(np.abs(ref).max() / rms))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--alg", choices=["iadm", "ftvcs"], default="iadm")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the n = 256 batched-vs-plain section")
    ap.add_argument("--batched-iters", type=int, default=300)
    ap.add_argument("--no-serving", action="store_true", help="skip the request-loop section")
    ap.add_argument("--serving-per", type=int, default=4,
                    help="matrices per (n, ratio) in the request-loop section (4: 36 matrices)")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the n = 512, m = 26214, B = 128 section (FP8 vs BF16 storage)")
    ap.add_argument("--large-iters", type=int, default=300)
    ap.add_argument("--no-dct", action="store_true", help="skip the partial-DCT section")
    ap.add_argument("--no-bb", action="store_true",
                    help="skip the n = 128 section of IADM with inner BB steps")
    # profiler modes: run one piece of the path and print one JSON line (no benchmark)
    ap.add_argument("--products", choices=sorted(PRODUCT_WORKLOADS), default=None,
                    help="only launch the two products of this workload `--reps` times each "
                         "(for rocprofv3), after a 256 MiB device copy that calibrates byte "
                         "counters")
    ap.add_argument("--storage", default="fp32",
                    choices=["fp32", "bf16", "bf16_split", "fp8_rowscale"])
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--form", choices=["fresh", "increment"], default="fresh",
                    help="form of the low-precision products for --products")
    ap.add_argument("--solve", choices=sorted(PRODUCT_WORKLOADS), default=None,
                    help="only solve `--batch` images of this workload with A in `--storage` "
                         "for `--iters` IADM iterations, once to warm up and once timed (for "
                         "rocprofv3), after the calibrating copy")
    ap.add_argument("--bb", type=int, default=1, metavar="J",
                    help="with --solve: J inner BB steps per IADM iteration (FP32 storage)")
    ap.add_argument("--dct-solve", type=int, default=0, metavar="N",
                    help="only solve a batch of `--batch` N x N partial-DCT problems for "
                         "`--iters` iterations (for rocprofv3)")
    args = ap.parse_args()
    if args.products or args.dct_solve or args.solve:
        profile_mode(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the method's images are "
                          "independent given A, so more GPUs only replicate A and split the "
                          "batch; run with --gpus 1"}), flush=True)
        sys.exit(2)

    import torch

    import oracle as O
    from paper_1001_1774_amd import synth, tvcs

    t0 = time.time()
    p = synth.workload("n128_m4096")            # FP64 A, FP64 f
    log(f"workload n128_m4096 generated in {time.time() - t0:.1f}s")
    tau = O.default_tau(p.A)
    flags_alg = tvcs.TVCS_IADM if args.alg == "iadm" else 0

    # ---- FP64 oracle on the host cores: full reconstructions of image 0, repeated
    # until about 10 s of CPU work (at most 30 s) -------------------------------
    cpu = None
    ref_u = None
    if not args.no_cpu_baseline:
        alg = O.iadm if args.alg == "iadm" else O.ftvcs
        runs, total = 0, 0.0
        while runs == 0 or (total < 10.0 and total * (runs + 1) / runs <= 30.0):
            t0 = time.perf_counter()
            ref = alg(p.A, p.f[:1], p.n, p.mu, p.beta, tau, tol=0, maxit=args.iters)
            total += time.perf_counter() - t0
            runs += 1
            if ref_u is None:
                ref_u = ref.u[0]
        cpu = {"value": runs / total, "unit": "reconstructions/s", "cores": cpu_threads(),
               "kind": "oracle",
               "sample": f"{runs} full reconstructions of image 0 ({args.iters} "
                         f"{args.alg.upper()} iterations each, FP64 numpy, {total:.1f} s)"}
        log(f"cpu oracle: {total / runs:.2f}s per reconstruction ({runs} runs)")

    # ---- GPU --------------------------------------------------------------------
    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    solver = tvcs.Solver(p.A.astype(np.float32), p.n, storage="fp32")
    solver.tau = tau
    h = solver.h
    f = torch.from_numpy(p.f[0].astype(np.float32)).to(dev)
    u = torch.empty(p.N, dtype=torch.float32, device=dev)
    st = tvcs.tvcs_stats()

    def step():
        rc = tvcs.tvcs_solve(h, f, p.mu, p.beta, 0.0, args.iters, flags_alg, u, None, st)
        if rc < 0:
            raise tvcs.TvcsError(rc, tvcs.tvcs_last_error())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    rec_s = args.steps / elapsed
    rel_err = psnr = None
    if ref_u is not None:
        ug = u.cpu().numpy().astype(np.float64).reshape(p.n, p.n)
        rel_err = float(np.linalg.norm(ug - ref_u) / np.linalg.norm(ref_u))
        psnr = psnr_db(ug, ref_u)

    # ---- roofline of the products (HIP events on the solver's stream) -------------
    ms_fwd, ms_adj = solver.time_products(B=1, reps=20)
    a_bytes = 4.0 * p.m * p.N
    fwd_bytes = a_bytes + 4.0 * (p.N + 2 * p.m)        # A, u, f, r
    adj_bytes = a_bytes + 4.0 * (p.m + p.N)            # A, r, g
    fwd_gbs = fwd_bytes / (ms_fwd * 1e-3) / 1e9
    adj_gbs = adj_bytes / (ms_adj * 1e-3) / 1e9

    # achievable peaks on this device (streaming read of 2 GiB, MFMA chains)
    peak_read, peak_mfma = tvcs.measure_peaks(2 << 30, 10)
    log(f"measured peaks: HBM read {peak_read:.0f} GB/s, bf16 MFMA {peak_mfma:.0f} TFLOP/s")
    ACHIEVABLE.update(hbm_read_gbs=peak_read, mfma_bf16_tflops=peak_mfma)

    # The solve's dominant kernel: one image at n = 128 takes both products in one
    # pass over A (k_gemv_fused; its band partials are then added by k_sum_bands);
    # the two separate products above are what a batch of images uses.
    ms_pass, ms_sum = solver.time_fused(reps=20)
    pass_bytes = a_bytes + 4.0 * (2 * p.N + p.m)        # A, u, f, g
    pass_gbs = pass_bytes / (ms_pass * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": pass_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": pass_gbs / HBM_PEAK_GBS, "traffic": measured_traffic("k_gemv_fused"),
                "algorithmic_bytes": pass_bytes,
                "kernel": "k_gemv_fused (g = A^T (A u - f), A read once)",
                "launch_ms": ms_pass, "band_sum_ms": ms_sum,
                "achievable_peak": peak_read, "frac_of_achievable": pass_gbs / peak_read}

    out = {
        "metric": "reconstructions/sec at <=1e-4 rel err vs FP64 (batched vs plain); GEMV GB/s",
        "value": rec_s,
        "unit": "reconstructions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"n128_m4096_fp32_{args.alg}{args.iters}", "n": p.n, "m": p.m,
                   "iterations": args.iters, "algorithm": args.alg.upper(), "storage": "fp32",
                   "mu": p.mu, "beta": p.beta, "tau": tau, "batch": 1, "seed_A": p.seed_A},
        "rel_err_vs_fp64_oracle": rel_err,
        "psnr_db_vs_fp64_oracle": psnr,
        "measured_peaks": dict(ACHIEVABLE),
        # the two products as separate passes (the path of batches of images)
        "gemv_gbs": {"forward": fwd_gbs, "adjoint": adj_gbs,
                     "forward_ms": ms_fwd, "adjoint_ms": ms_adj},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if not args.no_bb:
        out["bb_n128"] = bench_bb(np, torch, p, tau, solver)
    solver.close()
    del solver
    if not args.no_batched:
        out["batched_n256"] = bench_batched(args, np, torch, O, synth, tvcs)
        # the FP32 products where A (3.4 GB) is far larger than the 256 MB Infinity
        # Cache: an HBM rate, not a cache rate
        pf = out["batched_n256"]["plain_fp32"]
        out["gemv_hbm_n256"] = {
            "forward_gbs": pf["gemv_gbs_forward"], "adjoint_gbs": pf["gemv_gbs_adjoint"],
            "forward_frac": pf["gemv_gbs_forward"] / HBM_PEAK_GBS,
            "adjoint_frac": pf["gemv_gbs_adjoint"] / HBM_PEAK_GBS,
            "a_bytes": 4 * 13107 * 65536}
    if not args.no_serving:
        out["serving"] = bench_serving(args, np, synth, tvcs)
    if not args.no_large:
        out["large_n512"] = bench_large(args, np, torch, O, synth, tvcs)
    if not args.no_dct:
        out["partial_dct"] = bench_dct(args, np, torch, O, synth, tvcs)
    if "batched_n256" in out:
        # the metric's comparison: batched low-precision against the plain FP32 path at
        # n = 256, with the error against the FP64 oracle at the timed iteration count
        bn = out["batched_n256"]
        out["batched_vs_plain_n256"] = {
            k: {"rec_per_s": bn[k]["rec_per_s"], "speedup": bn[k]["speedup_vs_plain_fp32"],
                "max_rel_err_vs_fp64": max(e["rel_err"] for e in
                                           bn[k]["error_vs_fp64_oracle_fp64_A"].values()),
                "meets_1e-4": bn[k]["meets_1e-4"]} for k in ("bf16_split", "bf16")}
        out["batched_vs_plain_n256"]["plain_fp32_rec_per_s"] = bn["plain_fp32"]["rec_per_s"]
    print(json.dumps(out), flush=True)


PRODUCT_WORKLOADS = {"n128_m4096", "n256_m13107_b64", "n512_m26214_b128"}
COPY_BYTES = 256 << 20     # the plain copy that calibrates FETCH_SIZE / WRITE_SIZE


def profile_mode(args):
    """Launch one piece of the path for a profiler and print what it timed.

    --products W: the forward product (r = A u - f) and the adjoint product (A^T r)
    of workload W's A in `--storage`, for a batch of `--batch`, `--reps` launches
    each through tvcs_time_products (`--form increment`: the one-part increment form
    of the low-precision products); for one image with FP32 A at n*n <= 16384 also
    the one-pass product and its band sum (tvcs_time_fused).  First copies a 256 MiB device buffer once: a
    plain copy of known size (reads and writes 268435456 bytes) against which the
    FETCH_SIZE / WRITE_SIZE counters are scaled.
    --solve W: `--batch` images of workload W (its seeded images, repeated when the
    batch is larger) with A in `--storage`, IADM for `--iters` iterations, once to warm
    up and once timed (`--bb J`: with J inner BB steps per iteration).
    --dct-solve N: a batch of seeded N x N partial-DCT problems (30 % of the
    coefficients, IADM, mu = 500, beta = 2^6, tau = 1.9) solved for `--iters`
    iterations, once to warm up and once timed."""
    import torch

    from paper_1001_1774_amd import synth, tvcs
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if args.dct_solve:
        q = synth.make_dct_problem(f"dct{args.dct_solve}", args.dct_solve, 0.3, batch=args.batch)
        F = torch.from_numpy(q.f.astype(np.float32)).cuda()
        with tvcs.Solver.partial_dct(q.rows, q.n) as s:
            s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=args.iters, iadm=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=args.iters, iadm=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        print(json.dumps({"dct": args.dct_solve, "m": q.m, "batch": args.batch,
                          "iters": args.iters, "ms_per_iter": 1e3 * dt / args.iters}), flush=True)
        return
    if args.solve:
        p = synth.workload(args.solve, dtype=np.float32)
        F = torch.from_numpy(p.f[np.arange(args.batch) % p.B].astype(np.float32)).cuda()
        with tvcs.Solver(p.A, p.n, storage=args.storage) as s:
            s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=args.iters, iadm=True, bb_steps=args.bb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=args.iters, iadm=True,
                                bb_steps=args.bb)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tiles = s.tiles
        print(json.dumps({"workload": args.solve, "storage": args.storage, "batch": args.batch,
                          "iters": args.iters, "bb_steps": args.bb, "ms_per_iter": 1e3 * dt / args.iters,
                          "tiles": tiles, "fresh_iteration_fraction": fresh_fraction(out["stats"]),
                          "copy_bytes": COPY_BYTES}), flush=True)
        return
    p = synth.workload(args.products, batch=1, dtype=np.float32)
    with tvcs.Solver(p.A, p.n, storage=args.storage) as s:
        fwd, adj = s.time_products(args.batch, args.reps, increment=args.form == "increment")
        tiles = s.tiles
        # one image with FP32 A at n*n <= 16384: also the one-pass product and its
        # band sum (the kernels a single-image solve runs)
        fused = (s.time_fused(args.reps) if args.storage == "fp32" and args.batch == 1
                 and p.N <= 16384 else None)
    print(json.dumps({"workload": args.products, "storage": args.storage, "batch": args.batch,
                      "tiles": tiles,
                      "form": args.form, "reps": args.reps, "forward_ms": fwd,
                      "adjoint_ms": adj, "fused_pass_ms": fused[0] if fused else None,
                      "band_sum_ms": fused[1] if fused else None,
                      "copy_bytes": COPY_BYTES}), flush=True)


MFMA_BF16_PEAK = 2.5e15   # MI355X dense bf16 MFMA, FLOP/s
ACHIEVABLE = {}           # peaks measured on the device (filled in main)


def product_rates(storage, m, N, B, ms_f, ms_a, increment=False):
    """HBM and MFMA rates of the two batched products (HIP-event times per launch).
    Useful flops are 2 m N B per product; fresh products execute 2 bf16 MFMA
    products per useful one (batch operand split hi + lo), 3 with split storage of
    A; the increment form executes 1 (2 with split storage)."""
    elem = {"bf16": 2, "bf16_split": 4, "fp8_rowscale": 1}[storage]
    execd = (2 if storage == "bf16_split" else 1) if increment else \
        (3 if storage == "bf16_split" else 2)
    a_bytes = elem * m * N
    useful = 2.0 * m * N * B
    out = {"gemm_forward_ms": ms_f, "gemm_adjoint_ms": ms_a}
    for name, ms in (("forward", ms_f), ("adjoint", ms_a)):
        t = ms * 1e-3
        out[f"gemm_{name}_gbs"] = a_bytes / t / 1e9
        out[f"gemm_{name}_hbm_frac"] = a_bytes / t / (HBM_PEAK_GBS * 1e9)
        out[f"mfma_useful_frac_{name}"] = useful / t / MFMA_BF16_PEAK
        out[f"mfma_executed_frac_{name}"] = execd * useful / t / MFMA_BF16_PEAK
        if ACHIEVABLE:
            out[f"gemm_{name}_frac_of_achievable_hbm"] = a_bytes / t / (ACHIEVABLE["hbm_read_gbs"] * 1e9)
            out[f"mfma_executed_frac_of_achievable_{name}"] = (
                execd * useful / t / (ACHIEVABLE["mfma_bf16_tflops"] * 1e12))
    return out


def fresh_fraction(stats):
    """Share of the iterations whose products were fresh (the rest were increments)."""
    it = sum(st["iters"] for st in stats)
    return sum(st["fresh_iters"] for st in stats) / it if it else None


def bench_batched(args, np, torch, O, synth, tvcs):
    """n = 256, m = 13107 (20 %), 64 images sharing A: plain FP32 (one image per
    solve) against the batched MFMA path in split and plain BF16 storage, at the same
    number of IADM iterations.  Images 0 (noise 1e-3) and 45 (noise 1e-2) are checked
    against the FP64 oracle on the FP64 A at that iteration count.  The CPU baseline
    is the FP64 oracle on the whole batch (products as A @ U over the 64 images) for
    a bounded number of iterations, scaled to the timed count."""
    K = args.batched_iters
    t0 = time.time()
    sig = [1e-3 if i % 2 == 0 else 1e-2 for i in range(64)]
    p = synth.workload("n256_m13107_b64", sigma=sig)
    log(f"workload n256_m13107_b64 generated in {time.time() - t0:.1f}s")
    A32 = p.A.astype(np.float32)
    F = torch.from_numpy(p.f.astype(np.float32)).cuda()
    res = {"workload": "n256_m13107_b64", "n": p.n, "m": p.m, "batch": p.B, "iterations": K,
           "algorithm": "IADM", "seed_A": p.seed_A}
    tau = None
    # plain FP32: one image per solve
    with tvcs.Solver(A32, p.n, storage="fp32") as s:
        tau = s.tau
        s.solve(F[0], mu=p.mu, beta=p.beta, maxit=20, iadm=True)          # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(F[0], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms_f, ms_a = s.time_products(B=1, reps=10)
    gbs = 4.0 * p.m * p.N / 1e9
    res["plain_fp32"] = {"rec_per_s": 1.0 / dt, "ms_per_iter": 1e3 * dt / K,
                         "gemv_gbs_forward": gbs / (ms_f * 1e-3),
                         "gemv_gbs_adjoint": gbs / (ms_a * 1e-3)}
    log(f"plain fp32 n=256: {1e3 * dt / K:.3f} ms/iter")
    # FP64 oracle on images 0 and 45 at the timed iteration count
    sample = [0, 45]
    t0 = time.perf_counter()
    ref = O.iadm(p.A, p.f[sample], p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    log(f"oracle check ({len(sample)} images, {K} iterations): {time.perf_counter() - t0:.1f}s")
    for storage in ("bf16_split", "bf16"):
        with tvcs.Solver(A32, p.n, storage=storage) as s:
            s.tau = tau
            s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=10, iadm=True)    # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ms_f, ms_a = s.time_products(B=p.B, reps=10)
            mi_f, mi_a = s.time_products(B=p.B, reps=10, increment=True)
            tiles = s.tiles
        U = out["u"].cpu().numpy().astype(np.float64)
        errs = {}
        for j, b in enumerate(sample):
            d = U[b] - ref.u[j]
            errs[f"image{b}_sigma{sig[b]:g}"] = {
                "rel_err": float(np.linalg.norm(d) / np.linalg.norm(ref.u[j])),
                "max_rel_err": float(np.abs(d).max() / np.abs(ref.u[j]).max()),
                "psnr_db": psnr_db(U[b], ref.u[j])}
        res[storage] = {
            "rec_per_s": p.B / dt, "ms_per_iter": 1e3 * dt / K,
            "speedup_vs_plain_fp32": (p.B / dt) / res["plain_fp32"]["rec_per_s"],
            "error_vs_fp64_oracle_fp64_A": errs, "oracle_check_iterations": K,
            "meets_1e-4": all(e["rel_err"] <= 1e-4 for e in errs.values()),
            "fresh_iteration_fraction": fresh_fraction(out["stats"]),
            "fresh": product_rates(storage, p.m, p.N, p.B, ms_f, ms_a),
            "increment": product_rates(storage, p.m, p.N, p.B, mi_f, mi_a, increment=True),
            "tiles_autotuned": tiles,
        }
        log(f"{storage} B=64: {1e3 * dt / K:.3f} ms/iter, errors {[round(e['rel_err'], 8) for e in errs.values()]}")
    # FP64 oracle on the whole batch (the host's batched baseline), bounded iterations
    KC = 10
    t0 = time.perf_counter()
    O.iadm(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=KC)
    tc = time.perf_counter() - t0
    res["cpu_baseline"] = {
        "value": p.B / (tc * K / KC), "unit": "reconstructions/s", "cores": cpu_threads(),
        "kind": "oracle",
        "sample": f"FP64 oracle on all {p.B} images at once (A @ U products) for {KC} "
                  f"iterations ({tc:.1f} s), scaled to {K} iterations"}
    log(f"cpu oracle batched: {tc:.1f}s for {KC} iterations of {p.B} images")
    # the products' rates as the batch grows (bf16 storage, increment form): the
    # arithmetic intensity 2B / s_A moves the products from the HBM roofline towards
    # the MFMA one
    sweep = {}
    with tvcs.Solver(A32, p.n, storage="bf16") as s:
        for Bs in (64, 128, 256):
            ms_f, ms_a = s.time_products(B=Bs, reps=5, increment=True)
            r = product_rates("bf16", p.m, p.N, Bs, ms_f, ms_a, increment=True)
            r["tiles_autotuned"] = s.tiles
            ai = 2.0 * Bs / 2.0                           # useful flops per A byte
            bound = min(MFMA_BF16_PEAK, ai * HBM_PEAK_GBS * 1e9)
            r["roofline_bound_tflops"] = bound / 1e12
            r["roofline_bound"] = "mfma" if MFMA_BF16_PEAK < ai * HBM_PEAK_GBS * 1e9 else "hbm"
            r["frac_of_roofline_forward"] = 2.0 * p.m * p.N * Bs / (ms_f * 1e-3) / bound
            r["frac_of_roofline_adjoint"] = 2.0 * p.m * p.N * Bs / (ms_a * 1e-3) / bound
            sweep[f"B{Bs}"] = r
            log(f"bf16 increment products B={Bs}: {ms_f:.3f} / {ms_a:.3f} ms")
    res["bf16_increment_batch_sweep"] = sweep
    res["bb_split"] = bench_bb_batched(np, torch, tvcs, p, A32, F, tau)
    return res


def bench_bb_batched(np, torch, tvcs, p, A32, F, tau, J=3):
    """Split storage, all 64 images: IADM against IADM with J inner BB steps, as the
    distance of each image to the limit of the iteration (IADM + J BB steps after 1500
    outer iterations, 9000 products) after a given number of products with A, and the
    time to get there (median and largest distance over the images)."""
    with tvcs.Solver(A32, p.n, storage="bf16_split") as s:
        s.tau = tau

        def run(maxit, bb):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=maxit, iadm=True, bb_steps=bb)
            torch.cuda.synchronize()
            return r["u"].cpu().numpy().astype(np.float64), 1e3 * (time.perf_counter() - t0)

        run(5, J)
        ref, ms_ref = run(1500, J)
        nr = np.linalg.norm(ref.reshape(p.B, -1), axis=1)
        rows = []
        for bb, ks in ((1, (300, 900)), (J, (100, 150, 200, 300))):
            for k in ks:
                u, ms = run(k, bb)
                d = np.linalg.norm((u - ref).reshape(p.B, -1), axis=1) / nr
                rows.append({"method": "iadm" if bb == 1 else f"iadm_bb{J}", "outer_iters": k,
                             "a_products": 2 * k * bb, "ms": ms, "rec_per_s": p.B / (ms * 1e-3),
                             "median_dist_to_limit": float(np.median(d)),
                             "max_dist_to_limit": float(d.max())})
                log(f"bb split section: {rows[-1]}")
    return {"limit": f"IADM with {J} BB steps, 1500 outer iterations ({ms_ref:.0f} ms for "
                     f"{p.B} images)", "runs": rows}


def bench_serving(args, np, synth, tvcs):
    """Request loop: Poisson arrivals over resident BF16 matrices for n in {64, 128,
    256} and sampling ratios {0.1, 0.2, 0.3} (`--serving-per` matrices per pair),
    per-request tol in {1e-3, 1e-4} (cap 3000 iterations), IADM, mu = 1e3, beta = 10.
    First the saturated throughput (all requests at t = 0), then arrival rates of 0.5,
    0.8 and 0.95 of it.  The A-stream rate is the bytes of A the replays streamed
    over the wall time, against the HBM roofline."""
    from paper_1001_1774_amd import serving as S
    per = args.serving_per
    t0 = time.time()
    pools, solvers = [], []
    seed = 2001
    for n in (64, 128, 256):
        for r in (0.1, 0.2, 0.3):
            for _ in range(per):
                p = synth.make_problem(f"srv{seed}", n=n, ratio=r, batch=16, seed_A=seed,
                                       image_index0=100 * seed, dtype=np.float32)
                solvers.append(tvcs.Solver(p.A, n, storage="bf16"))
                pools.append(p.f.astype(np.float32))
                seed += 1
    log(f"serving: {len(solvers)} matrices ready in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(7)
    count = args.serving_requests

    def requests(rate):
        reqs = []
        for _ in range(count):
            mi = int(rng.integers(len(solvers)))
            reqs.append(S.Request(matrix=mi, f=pools[mi][int(rng.integers(16))],
                                  tol=float(rng.choice([1e-3, 1e-4])), maxit=3000))
        arr = S.poisson_arrivals(count, rate, int(rng.integers(1 << 30))) if rate else np.zeros(count)
        for r_, a in zip(reqs, arr):
            r_.arrival = float(a)
        return reqs

    keys = ("rec_per_s", "p50_ms", "p99_ms", "mean_iters", "a_stream_gbs", "wall_s")
    res = {"matrices": len(solvers), "storage": "bf16", "slots_per_matrix": 32,
           "requests_per_run": count, "algorithm": "IADM"}
    with S.Server(slots=32, mu=1e3, beta=10.0, iadm=True) as srv:
        for s_ in solvers:
            srv.add_matrix(s_)
        sat = S.run_arrivals(srv, requests(None))
        res["saturated"] = {k: sat[k] for k in keys}
        res["saturated"]["a_stream_frac_of_hbm"] = sat["a_stream_gbs"] / HBM_PEAK_GBS
        log(f"serving saturated: {sat['rec_per_s']:.1f} rec/s, A stream {sat['a_stream_gbs']:.0f} GB/s")
        for frac in (0.5, 0.8, 0.95):
            o = S.run_arrivals(srv, requests(frac * sat["rec_per_s"]))
            res[f"poisson_{frac}"] = {k: o[k] for k in keys}
            log(f"serving at {frac} of saturation: p50 {o['p50_ms']:.1f} ms, "
                f"p99 {o['p99_ms']:.1f} ms")
        res["device_bytes"] = srv.device_bytes
    for s_ in solvers:
        s_.close()
    return res


def bench_large(args, np, torch, O, synth, tvcs):
    """n = 512, m = 26214 (10 %), 128 images sharing A, IADM, 300 iterations:
    FP8-E4M3 with row scales against BF16 storage.  Images 5 and 100 are checked after
    KC iterations against the FP64 oracle on the matrix each format represents (the
    de-quantised A: the arithmetic's error) and on the FP64 A (the storage format's
    effect), as relative error and PSNR; the oracle run on the de-quantised A, held in
    host memory, is the CPU baseline, scaled to the timed count."""
    import threading
    t0 = time.time()
    p = synth.workload("n512_m26214_b128", dtype=np.float32)
    log(f"workload n512_m26214_b128 generated in {time.time() - t0:.1f}s")
    F = torch.from_numpy(p.f.astype(np.float32)).cuda()
    K, KC, sample = args.large_iters, 30, [5, 100]
    res = {"workload": "n512_m26214_b128", "n": p.n, "m": p.m, "batch": p.B, "iterations": K,
           "algorithm": "IADM", "oracle_check_iterations": KC, "oracle_check_images": sample}
    A = p.A
    p.A = None
    fs = p.f[sample].astype(np.float32).astype(np.float64)

    def dequantized(storage):
        out = np.empty(A.shape, np.float64)
        nxt, lock = [0], threading.Lock()

        def work():
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 256
                if i >= A.shape[0]:
                    return
                out[i:i + 256] = O.dequantized_A(A[i:i + 256], storage) if storage else A[i:i + 256]
        ths = [threading.Thread(target=work) for _ in range(min(16, len(os.sched_getaffinity(0))))]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        return out

    tau = {}
    for storage in ("fp8_rowscale", "bf16"):
        with tvcs.Solver(A, p.n, storage=storage) as s:
            tau[storage] = s.tau
            s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=10, iadm=True)     # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            chk = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=KC, iadm=True)["u"]
            Uc = chk.cpu().numpy()[sample].astype(np.float64)
            ms_f, ms_a = s.time_products(B=p.B, reps=5)
            mi_f, mi_a = s.time_products(B=p.B, reps=5, increment=True)
            tiles = s.tiles
        res[storage] = {"rec_per_s": p.B / dt, "ms_per_iter": 1e3 * dt / K,
                        "tiles_autotuned": tiles,
                        "fresh_iteration_fraction": fresh_fraction(out["stats"]),
                        "fresh": product_rates(storage, p.m, p.N, p.B, ms_f, ms_a),
                        "increment": product_rates(storage, p.m, p.N, p.B, mi_f, mi_a,
                                                   increment=True)}
        log(f"{storage} n=512 B=128: {1e3 * dt / K:.3f} ms/iter")
        t1 = time.perf_counter()
        Aq = dequantized(storage)
        td = time.perf_counter() - t1
        t1 = time.perf_counter()
        ref = O.iadm(Aq, fs, p.n, p.mu, p.beta, tau[storage], tol=0, maxit=KC)
        tc = time.perf_counter() - t1
        del Aq
        res[storage]["error_vs_fp64_oracle_dequantized_A"] = [
            {"image": b, "rel_err": float(np.linalg.norm(Uc[j] - ref.u[j]) / np.linalg.norm(ref.u[j])),
             "max_rel_err": float(np.abs(Uc[j] - ref.u[j]).max() / np.abs(ref.u[j]).max()),
             "psnr_db": psnr_db(Uc[j], ref.u[j])} for j, b in enumerate(sample)]
        res[storage]["cpu_baseline"] = {
            "value": len(sample) / (tc * K / KC), "unit": "reconstructions/s",
            "cores": cpu_threads(), "kind": "oracle",
            "sample": f"FP64 oracle on the de-quantised A (55 GB, in host memory, built in "
                      f"{td:.0f} s) for {len(sample)} images x {KC} iterations ({tc:.1f} s), "
                      f"scaled to {K} iterations"}
        res[storage]["_u_check"] = Uc
        log(f"{storage} oracle check: {tc:.1f}s")
    # the storage formats' effect: the oracle on the FP64 A (the FP32 copy, whose
    # rounding is 2^-24 relative) with the same tau per format
    A64 = dequantized(None)
    for storage in ("fp8_rowscale", "bf16"):
        ref = O.iadm(A64, fs, p.n, p.mu, p.beta, tau[storage], tol=0, maxit=KC)
        Uc = res[storage].pop("_u_check")
        res[storage]["error_vs_fp64_oracle_fp64_A"] = [
            {"image": b, "rel_err": float(np.linalg.norm(Uc[j] - ref.u[j]) / np.linalg.norm(ref.u[j])),
             "psnr_db": psnr_db(Uc[j], ref.u[j])} for j, b in enumerate(sample)]
    del A64
    res["fp8_vs_bf16_speedup"] = res["fp8_rowscale"]["rec_per_s"] / res["bf16"]["rec_per_s"]
    return res


def bench_bb(np, torch, p, tau, solver, J=3):
    """IADM against IADM with J inner BB / line-search steps on the u-subproblem, on
    the n = 128, m = 4096 FP32 problem: the distance to the limit of the iteration
    (BB for 4000 outer iterations, 24000 products) after a given number of products
    with A, and the time to get there."""
    f = p.f[0].astype(np.float32)

    def run(maxit, bb):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solver.solve(f, mu=p.mu, beta=p.beta, maxit=maxit, iadm=True, bb_steps=bb)
        torch.cuda.synchronize()
        return r["u"].cpu().numpy().astype(np.float64), 1e3 * (time.perf_counter() - t0)

    run(10, J)
    ref, ms_ref = run(4000, J)
    nr = np.linalg.norm(ref)
    rows = []
    for bb, ks in ((1, (500, 1500, 3000)), (J, (100, 200, 300, 400, 530, 700, 1000))):
        for k in ks:
            u, ms = run(k, bb)
            rows.append({"method": "iadm" if bb == 1 else f"iadm_bb{J}", "outer_iters": k,
                         "a_products": 2 * k * bb, "ms": ms,
                         "rel_err_vs_limit": float(np.linalg.norm(u - ref) / nr)})
            log(f"bb section: {rows[-1]}")
    out = {"limit": f"IADM with {J} BB steps, 4000 outer iterations ({ms_ref:.0f} ms)",
           "runs": rows}
    for thr in (1e-2, 1e-3, 1e-4):
        for meth in ("iadm", f"iadm_bb{J}"):
            hit = [r for r in rows if r["method"] == meth and r["rel_err_vs_limit"] <= thr]
            out[f"{meth}_to_{thr:g}"] = ({"a_products": hit[0]["a_products"], "ms": hit[0]["ms"]}
                                        if hit else None)
    return out


def dct_product_bytes(n, m, B):
    """Bytes each partial-DCT product moves per launch: every pass reads and writes
    one n x n FP32 array per image; the column pass also reads the coefficient map
    (4 n^2 bytes, shared by the batch) and f and writes r (forward), or reads r
    (adjoint)."""
    N = n * n
    fwd = B * (8.0 * N + 8.0 * N + 8.0 * m) + 4.0 * N
    adj = B * (4.0 * m + 4.0 * N + 8.0 * N) + 4.0 * N
    return fwd, adj


def bench_dct(args, np, torch, O, synth, tvcs):
    """The partial-DCT operator (Sec. 3.2): 30 % of the orthonormal 2-D DCT-II
    coefficients (the DC term and the rest uniformly at random), IADM with
    tau = 1.9, beta = 2^6, mu = 500.
      * 128 x 128, one image, tol = 5e-5 (the comparison setting): time, iterations
        and error against the ground truth; a fixed-iteration run against the oracle;
      * images of 128^2, 256^2, 450^2 (mixed-radix transforms) and 512^2 in batches:
        ms per iteration and the rate of the two products (HIP events, bytes per
        launch as in dct_product_bytes)."""
    res = {}
    p = synth.make_dct_problem("dct128_r30", 128, 0.3)
    f = torch.from_numpy(p.f[0].astype(np.float32)).cuda()
    K = 300
    with tvcs.Solver.partial_dct(p.rows, p.n) as s:
        s.solve(f, mu=p.mu, beta=p.beta, tol=5e-5, maxit=6000, iadm=True)    # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = s.solve(f, mu=p.mu, beta=p.beta, tol=5e-5, maxit=6000, iadm=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        u = out["u"].cpu().numpy().astype(np.float64)
        it = out["stats"]["iters"]
        fixed = s.solve(f, mu=p.mu, beta=p.beta, maxit=K, iadm=True)["u"].cpu().numpy()
    ref = O.iadm(O.PartialDCT(p.n, p.rows), p.f[:1].astype(np.float32).astype(np.float64),
                 p.n, p.mu, p.beta, p.tau, tol=0, maxit=K)
    res["n128_r30_tol5e-5"] = {
        "iterations": it, "seconds": dt, "ms_per_iter": 1e3 * dt / it,
        "rel_err_vs_truth": float(np.linalg.norm(u - p.ubar[0]) / np.linalg.norm(p.ubar[0])),
        f"rel_err_vs_fp64_oracle_{K}_iters": float(np.linalg.norm(fixed - ref.u[0]) /
                                                   np.linalg.norm(ref.u[0]))}
    log(f"partial DCT 128^2 tol 5e-5: {it} iterations in {dt * 1e3:.1f} ms")
    for n, B, Kb in ((128, 1, 500), (128, 64, 300), (256, 64, 200), (450, 16, 100),
                     (512, 16, 100), (512, 64, 100)):
        q = synth.make_dct_problem(f"dct{n}_b{B}", n, 0.3, batch=B)
        F = torch.from_numpy(q.f.astype(np.float32)).cuda()
        with tvcs.Solver.partial_dct(q.rows, n) as s:
            s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=10, iadm=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=Kb, iadm=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ms_f, ms_a = s.time_products(B=B, reps=20)
        bf, ba = dct_product_bytes(n, q.m, B)
        key = f"n{n}_b{B}"
        res[key] = {"m": q.m, "iterations": Kb, "ms_per_iter": 1e3 * dt / Kb,
                    "image_iters_per_s": B * Kb / dt, "rec_per_s_at_300_iters": B * Kb / dt / 300,
                    "forward_ms": ms_f, "adjoint_ms": ms_a,
                    "forward_gbs": bf / (ms_f * 1e-3) / 1e9, "adjoint_gbs": ba / (ms_a * 1e-3) / 1e9}
        log(f"partial DCT n={n} B={B}: {1e3 * dt / Kb:.3f} ms/iter, products "
            f"{ms_f * 1e3:.1f} / {ms_a * 1e3:.1f} us")
    return res


if __name__ == "__main__":
    main()
