"""Request loop for the continuous-batching server (cmcg_server_* in include/cmcg.h).

Replays a seeded arrival schedule in real time: every request is submitted once its arrival
time has passed, the server is stepped (each step advances all resident solves by one batched
launch and admits queued requests as memory and slots free up), and each request's latency is
measured from its arrival time to the step after which its result was available.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional


@dataclasses.dataclass
class Record:
    index: int
    name: str
    n: int
    omega: float
    arrival_s: float
    done_s: float
    latency_s: float
    state: int
    status: int
    iterations: int
    steps_per_period: int
    rel_residual: float
    grid_updates: float


def percentile(xs: List[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    s = sorted(xs)
    k = max(0, min(len(s) - 1, int(math.ceil(q / 100.0 * len(s))) - 1))
    return s[k]


def run(server, requests, precision: str = "fp32", tol: float = 1e-6, max_iter: int = 1000,
        clock: Callable[[], float] = time.perf_counter,
        sleep: Callable[[float], None] = time.sleep,
        on_event: Optional[Callable[[str], None]] = None):
    """Serve `requests` (a list of cmcg_inputs.Request sorted by arrival) on `server`.
    Returns (records, summary)."""
    order = sorted(range(len(requests)), key=lambda k: requests[k].arrival_s)
    t0 = clock()
    nxt = 0
    running: Dict[int, int] = {}
    records: List[Record] = []
    steps = 0
    peak_active = 0
    while nxt < len(order) or running:
        now = clock() - t0
        while nxt < len(order) and requests[order[nxt]].arrival_s <= now:
            k = order[nxt]
            rid = server.submit(requests[k].problem, precision=precision, tol=tol,
                                max_iter=max_iter)
            running[rid] = k
            nxt += 1
        if not running:
            sleep(max(0.0, requests[order[nxt]].arrival_s - (clock() - t0)))
            continue
        active, queued = server.step()
        steps += 1
        peak_active = max(peak_active, active)
        for rid in list(running):
            state, U, rep, st = server.poll(rid)
            if state in (2, -1):
                k = running.pop(rid)
                done = clock() - t0
                req = requests[k]
                rep = rep or {}
                records.append(Record(
                    index=k, name=req.problem.name, n=int(req.problem.n[0]),
                    omega=float(req.problem.omega), arrival_s=req.arrival_s, done_s=done,
                    latency_s=done - req.arrival_s, state=state, status=st,
                    iterations=int(rep.get("iterations", 0)),
                    steps_per_period=int(rep.get("steps_per_period", 0)),
                    rel_residual=float(rep.get("rel_residual", float("nan"))),
                    grid_updates=float(rep.get("grid_updates", 0.0))))
                if on_event:
                    on_event(f"done {k} n={req.problem.n[0]} latency {done - req.arrival_s:.2f}s "
                             f"iters {rep.get('iterations')}")
    makespan = clock() - t0
    lat = [r.latency_s for r in records]
    ok = [r for r in records if r.state == 2]
    summary = {
        "requests": len(records), "completed": len(ok),
        "failed": len(records) - len(ok),
        "converged": sum(1 for r in ok if r.status == 0),
        "makespan_s": makespan,
        "solves_per_s": len(ok) / makespan if makespan > 0 else float("nan"),
        "p50_latency_s": percentile(lat, 50) if lat else float("nan"),
        "p99_latency_s": percentile(lat, 99) if lat else float("nan"),
        "max_latency_s": max(lat) if lat else float("nan"),
        "server_steps": steps, "peak_active": peak_active,
        "grid_updates_per_s": sum(r.grid_updates for r in ok) / makespan if makespan > 0 else 0.0,
    }
    return records, summary
