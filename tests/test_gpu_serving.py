"""GPU tests of the continuous-batching request loop (tvcs_server_*)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1001_1774_amd import tvcs
    tvcs.lib()
    return tvcs


def make_mix(count, seed, problems, tols=(1e-3, 1e-4), maxit=300):
    from paper_1001_1774_amd.serving import Request
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        mi = int(rng.integers(len(problems)))
        p = problems[mi]
        b = int(rng.integers(p.B))
        reqs.append(Request(matrix=mi, f=p.f[b].astype(np.float32), tol=float(rng.choice(tols)),
                            maxit=maxit))
    return reqs


@pytest.fixture(scope="module")
def problems():
    return [synth.make_problem("s32", n=32, m=307, batch=6, seed_A=51, n_shapes=6),
            synth.make_problem("s64", n=64, m=819, batch=6, seed_A=52),
            synth.make_problem("s64b", n=64, m=1229, batch=6, seed_A=53)]


@pytest.mark.parametrize("iadm", [True, False], ids=["iadm", "ftvcs"])
def test_alone_equals_in_the_mix(T, problems, iadm):
    """Each request's result and iteration count are the same in the mix as alone: bit
    for bit for the MFMA-stored matrices; for the FP32 one (n = 32) a solve alone
    takes the one-pass product, whose sums run in another order, so there the
    results agree to rounding (within the FP32 bar of 1e-5)."""
    from paper_1001_1774_amd import serving as S
    storages = ["fp32", "bf16", "bf16_split"]
    solvers = [T.Solver(p.A, p.n, storage=st) for p, st in zip(problems, storages)]
    reqs = make_mix(40, 7, problems)
    arr = S.poisson_arrivals(len(reqs), rate=400.0, seed=3)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    with S.Server(slots=8, mu=1e3, beta=10.0, iadm=iadm) as srv:
        for s in solvers:
            srv.add_matrix(s)
        out = S.run_arrivals(srv, reqs, keep_results=True)
    say(f"  mix: {out['count']} requests, {out['rec_per_s']:.1f} rec/s, p50 {out['p50_ms']:.1f} ms,"
        f" p99 {out['p99_ms']:.1f} ms, mean iters {out['mean_iters']:.0f}")
    mism = 0
    for i, r in enumerate(reqs):
        u_mix, st_mix = out["results"][i]
        u_alone, st_alone = S.solve_alone(solvers[r.matrix], r, 1e3, 10.0, iadm)
        assert st_mix["iters"] == st_alone["iters"], (i, st_mix, st_alone)
        if storages[r.matrix] == "fp32":
            e = rel(u_mix.ravel(), u_alone.ravel().astype(np.float64))
            assert e <= 1e-5, (i, e)
        elif not np.array_equal(u_mix.ravel(), u_alone.ravel()):
            mism += 1
    say(f"  bitwise mismatches (MFMA storage): {mism} of {len(reqs)}")
    assert mism == 0
    for s in solvers:
        s.close()


def test_alone_equals_in_the_mix_at_request_sizes(T):
    """The serving mix's image sides: bf16 groups at n = 64 (30 %), 128 (20 %) and 256
    (10 %) running side by side; every request equals its solve alone (bitwise, same
    iteration count), with products in both forms (fresh and increment)."""
    from paper_1001_1774_amd import serving as S
    problems = [synth.make_problem("c64", n=64, ratio=0.3, batch=4, seed_A=61, dtype=np.float32),
                synth.make_problem("c128", n=128, ratio=0.2, batch=4, seed_A=62, dtype=np.float32),
                synth.make_problem("c256", n=256, ratio=0.1, batch=4, seed_A=63, dtype=np.float32)]
    solvers = [T.Solver(p.A, p.n, storage="bf16") for p in problems]
    reqs = make_mix(30, 17, problems, maxit=200)
    arr = S.poisson_arrivals(len(reqs), rate=300.0, seed=5)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    with S.Server(slots=16, mu=1e3, beta=10.0, iadm=True) as srv:
        for s in solvers:
            srv.add_matrix(s)
        out = S.run_arrivals(srv, reqs, keep_results=True)
    say(f"  mix: {out['count']} requests, {out['rec_per_s']:.1f} rec/s, p50 {out['p50_ms']:.1f} ms,"
        f" p99 {out['p99_ms']:.1f} ms, mean iters {out['mean_iters']:.0f}")
    mism, incr = 0, 0
    for i, r in enumerate(reqs):
        u_mix, st_mix = out["results"][i]
        u_alone, st_alone = S.solve_alone(solvers[r.matrix], r, 1e3, 10.0, True)
        assert st_mix["iters"] == st_alone["iters"], (i, st_mix, st_alone)
        assert st_mix["fresh_iters"] == st_alone["fresh_iters"], (i, st_mix, st_alone)
        incr += st_mix["iters"] - st_mix["fresh_iters"]
        if not np.array_equal(u_mix.ravel(), u_alone.ravel()):
            mism += 1
    say(f"  bitwise mismatches: {mism} of {len(reqs)}; increment-form iterations {incr}")
    assert mism == 0
    assert incr > 0
    for s in solvers:
        s.close()


def test_mix_matches_oracle(T, problems):
    """FP32 requests served in the mix agree with the FP64 oracle (same tau)."""
    from paper_1001_1774_amd import serving as S
    p = problems[0]
    with T.Solver(p.A, p.n, storage="fp32") as sol:
        tau = O.default_tau(p.A)
        sol.tau = tau
        reqs = [S.Request(matrix=0, f=p.f[b].astype(np.float32), tol=0.0, maxit=120,
                          arrival=0.002 * b) for b in range(p.B)]
        with S.Server(slots=4, mu=p.mu, beta=p.beta, iadm=True) as srv:
            srv.add_matrix(sol)
            out = S.run_arrivals(srv, reqs, keep_results=True)
        ref = O.iadm(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=120)
        for b in range(p.B):
            u = out["results"][b][0].astype(np.float64)
            e = rel(u, ref.u[b])
            assert out["results"][b][1]["iters"] == 120
            assert e <= 1e-5, (b, e)


def test_budget_admission(T, problems):
    """With room for one matrix's slots at a time, groups take turns and the
    counted device memory never exceeds the budget."""
    from paper_1001_1774_amd import serving as S
    sols = [T.Solver(problems[i].A, problems[i].n, storage="bf16") for i in (1, 2)]
    # measure the matrices' storage and one group's slots without a budget
    with S.Server(slots=16, mu=1e3, beta=10.0, iadm=True) as probe:
        for s in sols:
            probe.add_matrix(s)
        base = probe.device_bytes
        rid = probe.submit(0, problems[1].f[0], 1e-3, 20)
        probe.step()
        group = probe.device_bytes - base
        while probe.step():
            pass
        assert probe.result(rid, 64) is not None
    budget = base + group + group // 2      # room for one group of slots, not two
    say(f"  storage {base / 2**20:.1f} MiB, one group {group / 2**20:.2f} MiB")
    with S.Server(slots=16, mu=1e3, beta=10.0, iadm=True, hbm_budget=budget) as srv:
        for s in sols:
            srv.add_matrix(s)
        reqs = make_mix(30, 11, [problems[1], problems[2]], maxit=150)
        ids = [(srv.submit(r.matrix, r.f, r.tol, r.maxit), r) for r in reqs]
        peak = 0
        pending = len(ids)
        steps = 0
        while pending:
            pending = srv.step()
            peak = max(peak, srv.device_bytes)
            steps += 1
            assert steps < 10000
        for rid, r in ids:
            assert srv.result(rid, 64) is not None
    say(f"  budget {budget / 2**20:.1f} MiB, peak counted {peak / 2**20:.1f} MiB, steps {steps}")
    assert peak <= budget
    # a budget below one group's slots: the round reports ENOMEM instead of spinning
    with S.Server(slots=16, mu=1e3, beta=10.0, iadm=True, hbm_budget=base + group // 2) as srv:
        for s in sols:
            srv.add_matrix(s)
        srv.submit(0, problems[1].f[0], 1e-3, 20)
        with pytest.raises(T.TvcsError) as ei:
            srv.step()
        assert ei.value.code == T.TVCS_ENOMEM
    for s in sols:
        s.close()


def test_budget_wait_is_bounded(T, problems):
    """With room for one group, a matrix whose requests keep arriving does not hold
    the memory forever: a request for the other matrix is served within a bounded
    number of rounds (the resident group stops admitting after a few rounds of
    waiting, finishes what it holds and gives its slots back)."""
    from paper_1001_1774_amd import serving as S
    sols = [T.Solver(problems[i].A, problems[i].n, storage="bf16") for i in (1, 2)]
    with S.Server(slots=8, mu=1e3, beta=10.0, iadm=True) as probe:
        for s in sols:
            probe.add_matrix(s)
        base = probe.device_bytes
        rid = probe.submit(0, problems[1].f[0], 1e-3, 20)
        probe.step()
        group = probe.device_bytes - base
        while probe.step():
            pass
        assert probe.result(rid, 64) is not None
    budget = base + group + group // 2      # room for one group of slots, not two
    f0, f1 = problems[1].f.astype(np.float32), problems[2].f.astype(np.float32)
    with S.Server(slots=8, mu=1e3, beta=10.0, iadm=True, hbm_budget=budget) as srv:
        for s in sols:
            srv.add_matrix(s)
        ids0 = [srv.submit(0, f0[k % len(f0)], 0.0, 40) for k in range(8)]
        srv.step()                          # matrix 0 resident and running
        rid1 = srv.submit(1, f1[0], 0.0, 30)
        rounds = 0
        while srv.result(rid1, 64) is None:
            ids0.append(srv.submit(0, f0[rounds % len(f0)], 0.0, 40))   # never idle
            srv.step()
            rounds += 1
            # 4 rounds of waiting + 4 replays to finish matrix 0's slots + 3 replays
            # for the 30 iterations of the request, with room for early returns
            assert rounds <= 60, "request for matrix 1 still waiting"
        say(f"  matrix 1 served after {rounds} rounds while matrix 0 kept receiving requests")
        while srv.step():
            pass
        for rid in ids0:
            assert srv.result(rid, 64) is not None
    for s in sols:
        s.close()


def test_submit_errors(T, problems):
    from paper_1001_1774_amd import serving as S
    p = problems[0]
    with T.Solver(p.A, p.n) as sol, S.Server(slots=2) as srv:
        mid = srv.add_matrix(sol)
        with pytest.raises(T.TvcsError):
            srv.submit(mid + 5, p.f[0], 1e-3, 10)
        with pytest.raises(T.TvcsError):
            srv.submit(mid, p.f[0], -1.0, 10)
        with pytest.raises(T.TvcsError):
            srv.submit(mid, p.f[0], 1e-3, 0)
        with pytest.raises(T.TvcsError):
            srv.result(12345, p.n)
        assert T.tvcs_server_add_matrix(srv.s, sol.h) == T.TVCS_EINVAL   # registered twice
