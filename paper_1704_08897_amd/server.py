"""Serving front end over the library's continuous-batching engine.

``Server`` wraps ``bhx_engine_*`` (admission against an HBM budget and a slot
limit, a native worker thread that lets new requests join the running batch
at every iteration-chunk boundary).  ``serve_stream`` plays a list of
requests at given arrival times: requests that the engine cannot admit yet
wait in arrival order and are retried as earlier ones complete.  Latency is
measured from arrival to completion (host monotonic clock).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

from . import bhx


@dataclass
class Request:
    phi: object                 # device tensor (ny, nx) float64
    F: object                   # device tensor, in/out
    bc: int
    h: float
    tol: float
    arrival: float = 0.0        # seconds from the start of the stream
    tag: object = None


@dataclass
class Result:
    request: Request
    stats: dict
    t_arrival: float
    t_submit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 64,
                 precision: int = 0, chunk: int = 16, warm_start: int = 0):
        # warm_start=1: each request's F holds its first iterate at the unknown
        # nodes (e.g. the extension of the previous time step)
        self.opts = bhx.default_opts(precision=precision, chunk=chunk, warm_start=warm_start)
        self.engine = bhx.engine_create(device, hbm_budget, max_slots, self.opts)

    def submit(self, req: Request):
        """Returns the request id, or None if the engine cannot admit it now."""
        nx, ny = int(req.phi.shape[1]), int(req.phi.shape[0])
        s, rid = bhx.engine_submit(self.engine, req.phi, req.F, nx, ny, req.h, req.bc, req.tol)
        if s == bhx.BUSY:
            return None
        if s != bhx.OK:
            raise bhx.BhxError(s)
        return rid

    def poll(self):
        return bhx.engine_poll(self.engine)

    def inflight(self) -> int:
        return bhx.engine_inflight(self.engine)

    def close(self):
        if self.engine:
            bhx.engine_destroy(self.engine)
            self.engine = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_stream(server: Server, requests, on_done=None, idle_sleep: float = 2e-4,
                 stall_timeout: float = 120.0):
    """Submit each request at its arrival time (relative to now), keep the
    ones that do not fit in a FIFO, collect completions.  Returns the list of
    Result in completion order.  Raises TimeoutError if requests are in
    flight and none completes for `stall_timeout` seconds."""
    pending = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    waiting = []                      # arrived, not yet admitted (FIFO)
    live = {}                         # id -> (index, t_arrival, t_submit)
    results = []
    t0 = time.perf_counter()
    last_progress = t0
    nxt = 0
    while nxt < len(pending) or waiting or live:
        now = time.perf_counter() - t0
        if live and now + t0 - last_progress > stall_timeout:
            raise TimeoutError(f"{len(live)} requests in flight, none completed in "
                               f"{stall_timeout:.0f} s")
        while nxt < len(pending) and requests[pending[nxt]].arrival <= now:
            waiting.append((pending[nxt], t0 + requests[pending[nxt]].arrival))
            nxt += 1
        while waiting:
            i, ta = waiting[0]
            rid = server.submit(requests[i])
            if rid is None:
                break
            live[rid] = (i, ta, time.perf_counter())
            waiting.pop(0)
        done = server.poll()
        if done or not live:
            last_progress = time.perf_counter()
        for rid, st in done:
            i, ta, ts = live.pop(rid)
            r = Result(requests[i], st.as_dict(), ta, ts, ts + st.seconds)
            results.append(r)
            if on_done:
                on_done(r)
        if not done:
            if nxt < len(pending) and not waiting and not live:
                time.sleep(max(0.0, min(0.01, requests[pending[nxt]].arrival - now)))
            else:
                time.sleep(idle_sleep)
    return results
