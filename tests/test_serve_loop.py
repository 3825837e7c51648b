"""Host logic of the serving request loop, with a fake server (no GPU)."""
import dataclasses

import numpy as np
import pytest

from paper_1609_03488_amd.serve import replay


@dataclasses.dataclass
class Req:
    rid: int
    arrival_s: float
    work: int          # rounds needed
    size: int          # bytes


@dataclasses.dataclass
class Prob:
    op: object
    l: int
    q: list
    b: np.ndarray
    c: np.ndarray
    n_signal: int


class FakeServer:
    """Admits while slots and bytes allow; a request finishes after `work` steps."""

    def __init__(self, ws, slots):
        self.free, self.slots = ws, slots
        self.live = {}
        self.next = 1
        self.steps = 0
        self.order = []

    def submit(self, op, l, q, b, c):
        req = op
        if len(self.live) >= self.slots or req.size > self.free:
            return None
        t = self.next
        self.next += 1
        self.free -= req.size
        self.live[t] = [req, req.work]
        self.order.append(req.rid)
        return t

    def step(self, k):
        self.steps += 1
        for v in self.live.values():
            v[1] -= 1
        return sum(1 for v in self.live.values() if v[1] > 0)

    def poll(self, t):
        return 0 if self.live[t][1] > 0 else 1

    def finished(self):
        return [t for t, v in self.live.items() if v[1] <= 0]

    def fetch(self, t):
        req, _ = self.live.pop(t)
        self.free += req.size
        return np.zeros(3), None, None, {"status": 1, "iters": 10 * req.work}

    def close(self):
        pass


def _prob(req):
    return Prob(req, 0, [], np.zeros(1), np.zeros(1), 3)


def test_all_requests_complete_in_arrival_order_of_admission():
    reqs = [Req(i, 0.0, 1 + i % 3, 10) for i in range(20)]
    fake = {}

    def factory(ws, slots):
        fake["s"] = FakeServer(ws, slots)
        return fake["s"]

    res = replay(reqs, _prob, workspace_bytes=35, max_slots=8, server_factory=factory)
    assert res["completed"] == 20 and res["solved"] == 20
    assert fake["s"].order == list(range(20))         # FIFO admission
    assert res["refusals"] > 0                         # memory (35 bytes) forced waiting
    assert res["p50_s"] <= res["p99_s"]
    assert res["mean_iters"] == pytest.approx(10 * np.mean([r.work for r in reqs]))


def test_latency_counts_from_arrival():
    reqs = [Req(0, 0.0, 2, 1), Req(1, 0.05, 1, 1)]
    res = replay(reqs, _prob, workspace_bytes=10, max_slots=4,
                 server_factory=lambda ws, sl: FakeServer(ws, sl))
    lat = {c.rid: c.latency_s for c in res["completions"]}
    assert set(lat) == {0, 1}
    assert all(v >= 0 for v in lat.values())
    # the second request cannot complete before it arrives
    assert [c for c in res["completions"] if c.rid == 1][0].done_s >= 0.05
