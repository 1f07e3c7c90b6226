"""Serving loop: continuous admission of independent TPCG solves on one GPU.

One solve is a chain of latency-bound steps: its symmetric eigensolver
occupies one compute unit at a time and its GEMMs a few hundred workgroups
for microseconds, so a lone solve leaves most of the GPU idle.  The server
keeps `slots` solves in flight: each slot is a worker thread with its own
HIP stream (default priority) and library context (its own stream-ordered
memory pool), and a dispatcher admits waiting requests in arrival order as
soon as a slot is free and the request's estimated device footprint fits
the HBM budget.  A request builds its operator and right-hand side in its
slot's context, solves, copies the solution's Tucker data to the host if
asked, and releases its device memory.  The FD preconditioner depends only
on (n_el, p) (the parametric 1D matrices, the Appendix B data and the
exponential sum), so each slot builds it once per pair and keeps it.

HIP multiplexes the streams of a process onto GPU_MAX_HW_QUEUES hardware
queues (4 by default); each slot drives three streams (its solve's main
stream and two for the speculative ST-HOSVD modes), so set the variable to
16 or so before HIP initialises, or independent kernels of different slots
serialise in a shared queue (bench.py does).

Latency of a request = completion - arrival (queueing included); throughput
= completions / makespan.  Every kernel of the library is deterministic, so
a request's result does not depend on what else is in flight.
"""
from __future__ import annotations

import dataclasses
import queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    n_el: int
    p: int
    R: int            # Kronecker terms of the operator
    rank: int         # Tucker rank of the right-hand side
    seed: int
    arrival: float = 0.0   # seconds after the start of the run
    tol: float = 1e-6
    eps_min: float = 1e-8
    maxit: int = 1000
    arith: str = "f64"     # "f64" or "mixed" (tpcg_solve's precision rule)


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    start: float
    done: float
    iters: int = 0
    relres: float = float("nan")
    converged: bool = False
    rank: tuple = ()
    f32_applications: int = 0
    solution: Optional[tuple] = None   # (core, [U1, U2, U3]) on the host when kept
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def request_workload(req: Request):
    """The deformed-geometry recipe (weighted Kronecker terms, white-noise
    rhs) at the request's sizes and seeds."""
    import workloads as W
    return W.weighted_cp(req.n_el, req.p, req.R, req.rank, req.seed, req.seed + 1)


def estimate_bytes(req: Request) -> int:
    """Device footprint estimate of one solve: the truncation core Z and its
    mode-2 Gram partial products (q^3 doubles each, q <= n), the Gram
    eigen-workspaces, and the stacked factors of the operator and
    preconditioner outputs (R_A r and R_P r columns of n doubles)."""
    n = req.n_el + req.p - 2
    q = n
    return int(8 * (4 * q ** 3 + 40 * q * q + 4 * 32 * n * max(req.R, 22) * n))


def mixed_requests(count: int, seed: int, n_els=(64, 128), ps=(2, 3, 4), Rs=(3, 6, 9),
                   ranks=range(1, 11), eps_min: float = 1e-8, maxit: int = 1000, arith: str = "f64") -> List[Request]:
    """A seeded mix of requests (sizes drawn uniformly from the given sets)."""
    rng = np.random.default_rng(seed)
    ranks = list(ranks)
    out = []
    for i in range(count):
        out.append(Request(rid=i, n_el=int(rng.choice(n_els)), p=int(rng.choice(ps)), R=int(rng.choice(Rs)),
                           rank=int(rng.choice(ranks)), seed=seed + 1 + 2 * i, eps_min=eps_min, maxit=maxit,
                           arith=arith))
    return out


def poisson_arrivals(requests: List[Request], rate: float, seed: int) -> List[Request]:
    """Copies of the requests with exponential inter-arrival gaps of mean
    1/rate (rate <= 0: all arrive at time 0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in requests:
        if rate > 0:
            t += rng.exponential(1.0 / rate)
        out.append(dataclasses.replace(r, arrival=t if rate > 0 else 0.0))
    return out


class _Slot:
    """A worker: one HIP stream, one library context and its preconditioners."""

    def __init__(self, device: int):
        import torch
        from . import tk
        self.stream = torch.cuda.Stream(device=device)   # default priority
        self.ctx = tk.Context(device, stream=self.stream.cuda_stream)
        self.precs = {}   # (n_el, p) -> Preconditioner

    def preconditioner(self, w):
        from . import problem
        key = (w.n_el, w.p)
        if key not in self.precs:
            self.precs[key] = problem.preconditioner(self.ctx, w)
        return self.precs[key]

    def close(self):
        self.precs.clear()
        self.ctx.close()


def library_solve(slot: _Slot, req: Request, keep: bool) -> dict:
    """Build the request's problem in the slot's context and solve it."""
    from . import problem, tk
    w = request_workload(req)
    ctx = slot.ctx
    op = problem.operator(ctx, w)
    P = slot.preconditioner(w)
    f = problem.rhs(ctx, w)
    x, info = tk.tpcg_solve(ctx, op, P, f, tol=req.tol, eps_min=req.eps_min, maxit=req.maxit, arith=req.arith,
                            allow_noconv=True)
    out = {"iters": info["iters"], "relres": info["relres"], "converged": bool(info["converged"]),
           "rank": tuple(info["rank"]), "f32_applications": info["f32_applications"]}
    if keep:
        out["solution"] = x.plain()
    ctx.sync()
    del x, op, f
    return out


class Server:
    """`slots` concurrent solves, admitted in arrival order within
    `hbm_budget` bytes of estimated footprint.  `solve` is the per-request
    work (library_solve by default; a stand-in in the host-logic tests)."""

    def __init__(self, slots: int = 8, hbm_budget: float = 128e9, device: int = 0,
                 solve: Optional[Callable] = None, make_slot: Optional[Callable] = None):
        self.n_slots = slots
        self.hbm_budget = hbm_budget
        self.solve = solve or library_solve
        make_slot = make_slot or (lambda: _Slot(device))
        self.slots = [make_slot() for _ in range(slots)]

    def close(self):
        for s in self.slots:
            if hasattr(s, "close"):
                s.close()

    def run(self, requests: List[Request], keep_solutions: bool = False) -> List[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if estimate_bytes(r) > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs more than the HBM budget on its own")
        free_slots: "queue.Queue[int]" = queue.Queue()
        for i in range(self.n_slots):
            free_slots.put(i)
        budget_lock = threading.Condition()
        in_use = [0.0]
        results: List[Result] = []
        res_lock = threading.Lock()
        threads = []
        t0 = time.perf_counter()

        def work(slot_id: int, r: Request, start: float):
            try:
                out = self.solve(self.slots[slot_id], r, keep_solutions)
                res = Result(r.rid, r.arrival, start, time.perf_counter() - t0, **out)
            except Exception as exc:  # reported per request, the server keeps running
                res = Result(r.rid, r.arrival, start, time.perf_counter() - t0, error=repr(exc))
            with res_lock:
                results.append(res)
            with budget_lock:
                in_use[0] -= estimate_bytes(r)
                budget_lock.notify_all()
            free_slots.put(slot_id)

        for r in reqs:
            now = time.perf_counter() - t0
            if r.arrival > now:
                time.sleep(r.arrival - now)
            need = estimate_bytes(r)
            with budget_lock:
                while in_use[0] + need > self.hbm_budget:
                    budget_lock.wait()
                in_use[0] += need
            slot_id = free_slots.get()
            th = threading.Thread(target=work, args=(slot_id, r, time.perf_counter() - t0), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        return sorted(results, key=lambda x: x.rid)


def summarize(results: List[Result]) -> dict:
    """Throughput (completions / makespan, from the first arrival) and latency
    percentiles of a run."""
    ok = [r for r in results if r.error is None]
    if not ok:
        return {"completed": 0, "errors": len(results)}
    t_first = min(r.arrival for r in results)
    makespan = max(r.done for r in ok) - t_first
    lat = np.array([r.latency for r in ok])
    return {"completed": len(ok), "errors": len(results) - len(ok), "makespan_s": makespan,
            "solves_per_s": len(ok) / makespan if makespan > 0 else float("inf"),
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                           "max": float(lat.max() * 1e3)},
            "converged": int(sum(r.converged for r in ok)),
            "iters_mean": float(np.mean([r.iters for r in ok])),
            "relres_max": float(max(r.relres for r in ok)),
            "f32_applications": int(sum(r.f32_applications for r in ok))}
