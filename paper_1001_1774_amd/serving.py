"""Driver for the native continuous-batching request loop (tvcs_server_* in the C ABI).

`Server` wraps the C calls; `run_arrivals` replays a list of requests against it
with given arrival times (e.g. Poisson) and reports latency percentiles and
throughput.  All scheduling (slot admission, HBM budget, per-matrix streams,
retirement) happens in the library; this module only submits, steps and collects.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import tvcs as T


class Server:
    def __init__(self, slots=64, mu=1e3, beta=10.0, iadm=True, hbm_budget=0):
        self.s = T.tvcs_server_create(hbm_budget, slots, mu, beta, T.TVCS_IADM if iadm else 0)
        if not self.s:
            raise T.TvcsError(T.TVCS_EINVAL, T.tvcs_last_error())
        self.n_of = {}
        self._keep = []

    def add_matrix(self, solver: "T.Solver") -> int:
        mid = T.tvcs_server_add_matrix(self.s, solver.h)
        if mid < 0:
            raise T.TvcsError(mid, T.tvcs_last_error())
        self.n_of[mid] = solver.n
        self._keep.append(solver)
        return mid

    def submit(self, matrix, f, tol, maxit) -> int:
        f = np.ascontiguousarray(f, dtype=np.float32)
        rid = T.tvcs_server_submit(self.s, matrix, f, tol, maxit)
        if rid < 0:
            raise T.TvcsError(rid, T.tvcs_last_error())
        return rid

    def step(self) -> int:
        rc = T.tvcs_server_step(self.s)
        if rc < 0:
            raise T.TvcsError(rc, T.tvcs_last_error())
        return rc

    def result(self, rid, n):
        u = np.empty(n * n, np.float32)
        st = T.tvcs_stats()
        rc = T.tvcs_server_result(self.s, rid, u, st)
        if rc < 0:
            raise T.TvcsError(rc, T.tvcs_last_error())
        if rc == 0:
            return None
        return u.reshape(n, n), dict(iters=st.iters, status=st.status,
                                     rel_change=st.rel_change, ms=st.ms,
                                     fresh_iters=st.fresh_iters)

    @property
    def device_bytes(self):
        return T.tvcs_server_device_bytes(self.s)

    @property
    def a_bytes(self):
        """Bytes of A the replays launched so far stream (tvcs_server_a_bytes)."""
        return T.tvcs_server_a_bytes(self.s)

    def close(self):
        if getattr(self, "s", None):
            T.tvcs_server_destroy(self.s)
            self.s = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class Request:
    matrix: int
    f: np.ndarray
    tol: float
    maxit: int
    arrival: float = 0.0      # seconds after the start of the run


def poisson_arrivals(count, rate, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def run_arrivals(server: Server, requests, keep_results=False):
    """Submit each request at its arrival time (relative to the start), step the
    server until all have finished; latency = finish - arrival."""
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    inflight = {}
    lat = np.zeros(len(requests))
    iters = np.zeros(len(requests), dtype=np.int64)
    results = {} if keep_results else None
    a0 = server.a_bytes
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    while done < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(order) and requests[order[nxt]].arrival <= now:
            i = order[nxt]
            r = requests[i]
            inflight[server.submit(r.matrix, r.f, r.tol, r.maxit)] = i
            nxt += 1
        if not inflight:
            if nxt < len(order):
                time.sleep(max(0.0, requests[order[nxt]].arrival - now))
            continue
        server.step()
        tnow = time.perf_counter() - t0
        for rid in list(inflight):
            i = inflight[rid]
            out = server.result(rid, server.n_of[requests[i].matrix])
            if out is None:
                continue
            del inflight[rid]
            lat[i] = tnow - requests[i].arrival
            iters[i] = out[1]["iters"]
            if keep_results:
                results[i] = out
            done += 1
    wall = time.perf_counter() - t0
    a_gbs = (server.a_bytes - a0) / wall / 1e9
    return dict(count=len(requests), wall_s=wall, rec_per_s=len(requests) / wall,
                a_stream_gbs=a_gbs,
                p50_ms=1e3 * float(np.percentile(lat, 50)),
                p99_ms=1e3 * float(np.percentile(lat, 99)),
                mean_iters=float(iters.mean()), latencies=lat, results=results)


def solve_alone(solver: "T.Solver", r: Request, mu, beta, iadm):
    """The same request through an ordinary single-image solve (for comparisons)."""
    out = solver.solve(r.f.astype(np.float32), mu=mu, beta=beta, tol=r.tol, maxit=r.maxit,
                       iadm=iadm)
    return out["u"].cpu().numpy(), out["stats"]


__all__ = ["Server", "Request", "poisson_arrivals", "run_arrivals", "solve_alone"]
