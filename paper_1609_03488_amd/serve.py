"""Request loop over the continuous-batching server (cgs_server_*).

Requests arrive on a trace clock; each arrival is admitted as soon as a slot is
free and its device footprint fits in the server's unused workspace; admitted
problems advance together (one launch per kernel for all of them) and leave as
soon as their own termination test passes.  Latency = completion time minus
arrival time.  All numerical work happens in libcgs.so.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from ._lib import Server, Settings, FP32
from .problems import ConeProblem


@dataclasses.dataclass
class Completed:
    rid: int
    arrival_s: float
    admitted_s: float
    done_s: float
    status: int
    iters: int
    x: Optional[np.ndarray]

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def replay(requests: Sequence, make_problem: Callable[[object], ConeProblem], *,
           settings: Optional[Settings] = None, workspace_bytes: int = 8 << 30,
           max_slots: int = 4096, steps_per_call: int = 10, keep_x: bool = False,
           time_scale: float = 1.0, stream=None, log: Optional[Callable[[str], None]] = None,
           server_factory: Optional[Callable[..., object]] = None) -> Dict[str, object]:
    """Replay `requests` (objects with .rid and .arrival_s, sorted by arrival).

    `make_problem(req)` builds the request's cone problem (host side, done when
    the request arrives).  Returns throughput, latency percentiles and the list
    of completions.
    """
    if server_factory is None:
        st = settings if settings is not None else Settings.make(precision=FP32)
        server = Server(workspace_bytes, max_slots, st, stream=stream)
    else:
        server = server_factory(workspace_bytes, max_slots)
    pending = collections.deque(requests)
    queued: collections.deque = collections.deque()   # arrived, waiting for memory / a slot
    running: Dict[int, tuple] = {}                     # ticket -> (req, problem, admitted time)
    done: List[Completed] = []
    refused = 0
    t0 = time.perf_counter()
    next_log = 1.0

    def now() -> float:
        return (time.perf_counter() - t0) / time_scale

    while pending or queued or running:
        t = now()
        while pending and pending[0].arrival_s <= t:
            req = pending.popleft()
            queued.append((req, make_problem(req)))
        while queued:
            req, pr = queued[0]
            ticket = server.submit(pr.op, pr.l, pr.q, pr.b, pr.c)
            if ticket is None:
                refused += 1
                break
            queued.popleft()
            running[ticket] = (req, pr, now())
        if not running:
            if pending:
                time.sleep(max(0.0, (pending[0].arrival_s - now()) * time_scale))
            continue
        server.step(steps_per_call)
        tdone = now()
        for ticket in server.finished():
            if ticket in running:
                req, pr, tadm = running.pop(ticket)
                x, _, _, info = server.fetch(ticket)
                done.append(Completed(req.rid, req.arrival_s, tadm, tdone, info["status"],
                                      info["iters"], x[:pr.n_signal].copy() if keep_x else None))
        if log is not None and tdone >= next_log:
            log(f"t={tdone:.1f}s done={len(done)} running={len(running)} queued={len(queued)} "
                f"pending={len(pending)}")
            next_log = tdone + 1.0
    wall = now()
    server.close()
    lat = np.array([c.latency_s for c in done])
    return {
        "completed": len(done),
        "wall_s": wall,
        "solves_per_s": len(done) / wall if wall > 0 else 0.0,
        "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_iters": float(np.mean([c.iters for c in done])) if done else None,
        "refusals": refused,
        "solved": int(sum(1 for c in done if c.status == 1)),
        "completions": done,
    }
