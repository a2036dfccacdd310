"""Admission order of the serving front end (CPU: a stand-in engine with a
byte budget, no GPU).  Later arrivals that fit are admitted past a blocked
oldest request, and an ageing bound stops that once the oldest has waited
long enough, so it is not starved."""
import time
from dataclasses import dataclass

import pytest

from paper_1704_08897_amd.server import Request, serve_stream


@dataclass
class _St:
    seconds: float
    status: int = 0

    def as_dict(self):
        return {"status": self.status, "seconds": self.seconds, "iterations": 1}


class FakeEngine:
    """Admits a request when its size fits the free budget; each request
    finishes `service` seconds after admission."""

    def __init__(self, budget, service):
        self.free = budget
        self.service = service
        self.live = {}
        self.next = 1
        self.admitted = []                     # tags in admission order

    def submit(self, req):
        size = req.tag[1]
        if size > self.free:
            return None
        self.free -= size
        rid = self.next
        self.next += 1
        self.live[rid] = (time.perf_counter(), size)
        self.admitted.append(req.tag[0])
        return rid

    def poll(self):
        now = time.perf_counter()
        out = []
        for rid, (t, size) in list(self.live.items()):
            if now - t >= self.service:
                del self.live[rid]
                self.free += size
                out.append((rid, _St(now - t)))
        return out


def _reqs(spec):
    # spec: (name, size, arrival)
    return [Request(None, None, 0, 1.0, 1e-8, arrival=a, tag=(n, s)) for n, s, a in spec]


def test_small_request_passes_blocked_large_one():
    # A occupies 6 of 10; B (8) cannot fit until A ends; C (3) fits now
    eng = FakeEngine(10, service=0.15)
    res = serve_stream(eng, _reqs([("A", 6, 0.0), ("B", 8, 0.01), ("C", 3, 0.02)]),
                       max_bypass_s=1.0)
    assert len(res) == 3
    assert eng.admitted == ["A", "C", "B"]
    lat = {r.request.tag[0]: r.latency for r in res}
    assert lat["C"] < 0.25                     # not held behind B


def test_strict_order_without_bypass():
    eng = FakeEngine(10, service=0.15)
    serve_stream(eng, _reqs([("A", 6, 0.0), ("B", 8, 0.01), ("C", 3, 0.02)]), max_bypass_s=0)
    assert eng.admitted == ["A", "B", "C"]


def test_ageing_bound_stops_bypass():
    """A stream of small requests keeps the budget busy; the large one would
    never fit if they kept passing it.  After max_bypass_s it is admitted
    next."""
    eng = FakeEngine(10, service=0.1)
    spec = [("A", 6, 0.0), ("B", 9, 0.005)]
    spec += [(f"s{i}", 3, 0.01 + 0.02 * i) for i in range(40)]
    res = serve_stream(eng, _reqs(spec), max_bypass_s=0.2)
    assert len(res) == len(spec)
    order = eng.admitted
    b = order.index("B")
    # some small requests passed B, but not all of them
    assert 0 < b < len(order) - 5
    waited = {r.request.tag[0]: r.t_submit - r.t_arrival for r in res}
    assert waited["B"] < 0.2 + 0.1 + 0.1       # bound + one service time + slack
