"""Serving front end over the library's continuous-batching engine.

``Server`` wraps ``bhx_engine_*`` (admission against an HBM budget and a slot
limit, a native worker thread that lets new requests join the running batch
at every iteration-chunk boundary).  ``serve_stream`` plays a list of
requests at given arrival times and collects completions.  Latency is
measured from arrival to completion (host monotonic clock).

Admission order.  Arrived requests wait in arrival order.  When the oldest
cannot be admitted (its workspace does not fit the free budget, or no slot is
free), later arrivals that do fit are admitted past it, so one large request
does not hold back smaller ones behind it.  An ageing bound keeps that from
starving the large one: once the oldest waiting request has waited
``max_bypass_s`` seconds, nothing is admitted past it until it is in, so the
capacity that completions free goes to it.
"""
from __future__ import annotations

import sys
import time
from dataclasses import dataclass

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
    """One engine on one device.  ``opts`` are ``bhx_opts`` fields applied to
    every request (precision, accurate, tol_inner, warm_start, ...);
    ``chunk`` is the number of iterations between admission points."""

    is_engine = True

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 64,
                 precision: int = 0, chunk: int = 16, warm_start: int = 0, **opts):
        # warm_start=1: each request's F holds its first iterate at the unknown
        # nodes (e.g. the extension of the previous time step)
        self.opts = bhx.default_opts(precision=precision, chunk=chunk, warm_start=warm_start,
                                     **opts)
        self.engine = bhx.engine_create(device, hbm_budget, max_slots, self.opts)
        self._key = bhx._register(self)

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
        """Stop the worker after the requests in flight finish and free the
        engine (idempotent)."""
        if self.engine:
            e, self.engine = self.engine, None
            bhx._open.pop(self._key, None)
            bhx.engine_destroy(e)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass


def serve_stream(server: Server, requests, on_done=None, idle_sleep: float = 2e-4,
                 stall_timeout: float = 120.0, max_bypass_s: float = 1.0,
                 lookahead: int = 64):
    """Submit each request at its arrival time (relative to now) and collect
    completions; returns the list of Result in completion order.

    Requests that cannot be admitted yet wait in arrival order.  While the
    oldest of them cannot be admitted, up to ``lookahead`` later ones are
    tried, and those that fit are admitted past it, unless the oldest has
    waited ``max_bypass_s`` seconds or more (then it alone is retried until
    it is in).  ``max_bypass_s=0`` gives strict arrival order.  Raises
    TimeoutError if requests are in flight and none completes for
    ``stall_timeout`` seconds."""
    pending = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    waiting = []                      # arrived, not yet admitted, arrival order
    live = {}                         # id -> (index, t_arrival, t_submit)
    results = []
    t0 = time.perf_counter()
    last_progress = t0
    nxt = 0

    def admit(pos):
        i, ta = waiting[pos]
        rid = server.submit(requests[i])
        if rid is None:
            return False
        live[rid] = (i, ta, time.perf_counter())
        waiting.pop(pos)
        return True

    while nxt < len(pending) or waiting or live:
        tnow = time.perf_counter()
        now = tnow - t0
        if live and tnow - last_progress > stall_timeout:
            raise TimeoutError(f"{len(live)} requests in flight, none completed in "
                               f"{stall_timeout:.0f} s")
        while nxt < len(pending) and requests[pending[nxt]].arrival <= now:
            waiting.append((pending[nxt], t0 + requests[pending[nxt]].arrival))
            nxt += 1
        while waiting and admit(0):
            pass
        if waiting and max_bypass_s > 0 and tnow - waiting[0][1] < max_bypass_s:
            pos = 1
            while pos < len(waiting) and pos <= lookahead:
                if not admit(pos):
                    pos += 1
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
