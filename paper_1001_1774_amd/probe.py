"""Run only the two dense products of a workload, or one partial-DCT solve, for profilers.

    python -m paper_1001_1774_amd.probe --workload n128_m4096 --storage fp32 --batch 1 --reps 5
    python -m paper_1001_1774_amd.probe --dct 512 --batch 64 --iters 40

First copies a 256 MiB device buffer once (a plain copy of known size: reads and
writes 268435456 bytes), which calibrates hardware byte counters such as
FETCH_SIZE / WRITE_SIZE; then launches the forward product (r = A u - f) and the
adjoint product (A^T r) `reps` times each through tvcs_time_products and prints
the HIP-event times.  With --dct n: a batch of seeded partial-DCT problems (30 % of
the coefficients, IADM, mu = 500, beta = 2^6, tau = 1.9) solved for `iters`
iterations, once to warm up and once timed.  Inputs are the seeded synthetic
workloads.
"""
import argparse
import json

import numpy as np
import torch

from . import synth, tvcs

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="n128_m4096", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--storage", default="fp32", choices=sorted(tvcs.STORAGE))
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--dct", type=int, default=0, help="image side of a partial-DCT solve")
    ap.add_argument("--iters", type=int, default=40)
    args = ap.parse_args()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if args.dct:
        dct_solve(args)
        return
    p = synth.workload(args.workload, batch=1, dtype=np.float32)
    with tvcs.Solver(p.A, p.n, storage=args.storage) as s:
        fwd, adj = s.time_products(args.batch, args.reps)
    print(json.dumps({"workload": args.workload, "storage": args.storage, "batch": args.batch,
                      "reps": args.reps, "forward_ms": fwd, "adjoint_ms": adj,
                      "copy_bytes": COPY_BYTES}), flush=True)


def dct_solve(args):
    import time
    q = synth.make_dct_problem(f"dct{args.dct}", args.dct, 0.3, batch=args.batch)
    F = torch.from_numpy(q.f.astype(np.float32)).cuda()
    with tvcs.Solver.partial_dct(q.rows, q.n) as s:
        s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=args.iters, iadm=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve_batch(F, mu=q.mu, beta=q.beta, maxit=args.iters, iadm=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    print(json.dumps({"dct": args.dct, "m": q.m, "batch": args.batch, "iters": args.iters,
                      "ms_per_iter": 1e3 * dt / args.iters}), flush=True)


if __name__ == "__main__":
    main()
