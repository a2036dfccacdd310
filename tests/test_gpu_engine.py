"""Serving engine on the GPU: continuous batching through the C interface.

A request's result must not depend on what else is in flight: the engine
keeps each request's work split (tiles, row groups) a function of its own
size, every reduction in a fixed order, and each request's scalars apart, so
a result in the mix is bit-identical to the same request solved alone.
"""
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_1704_08897_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08897_amd import bhx  # noqa: E402
from paper_1704_08897_amd.server import Request, Server, serve_stream  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def mixed_requests(count, seed=7, nmin=40, nmax=140, tol=1e-12):
    specs = W.request_stream(count, seed=seed, nmin=nmin, nmax=nmax, tol=tol)
    return [s.materialise() for s in specs]


@pytest.fixture(scope="module")
def handle():
    h = bhx.Handle(0)
    yield h
    h.close()


def alone(handle, p):
    """The request solved alone with bhx_extend_ex on the plan-table kernels,
    the family the engine runs (a single solve of a compile-time shape would
    otherwise take the shape instances, which agree only to rounding), with
    the engine's work-item policy (rows = -1: the fullest items)."""
    old = os.environ.get("BHX_SHAPE_KERNELS")
    os.environ["BHX_SHAPE_KERNELS"] = "0"
    try:
        F = dev(p.F)
        s, st = bhx.extend_ex(handle, dev(p.phi), F, bc=p.bc, h=p.h, tol=p.tol,
                              opts=bhx.default_opts(rows=-1))
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["BHX_SHAPE_KERNELS"]
        else:
            os.environ["BHX_SHAPE_KERNELS"] = old
    return s, st, F.cpu().numpy()


def test_mix_equals_alone(handle):
    probs = mixed_requests(6)
    srv = Server(0, hbm_budget=1 << 30, max_slots=8)
    try:
        reqs = [Request(dev(p.phi), dev(p.F), p.bc, p.h, p.tol, arrival=0.0) for p in probs]
        res = serve_stream(srv, reqs)
    finally:
        srv.close()
    assert len(res) == len(probs)
    for r in res:
        assert r.stats["status"] == bhx.OK, r.stats
    torch.cuda.synchronize()
    for p, q in zip(probs, reqs):
        s, st, ref_alone = alone(handle, p)
        got = q.F.cpu().numpy()
        assert np.array_equal(got, ref_alone)
        ref, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
        assert O.relative_l2(got, ref) <= 1e-9


def test_large_requests_mix_equals_alone(handle):
    """Requests large enough that the engine's transform lists hold more
    items than its persistent grids have blocks (each block takes several
    items of different requests): each result still equals the request
    solved alone bit for bit."""
    probs = mixed_requests(5, seed=13, nmin=380, nmax=700, tol=1e-10)
    srv = Server(0, hbm_budget=4 << 30, max_slots=8)
    try:
        reqs = [Request(dev(p.phi), dev(p.F), p.bc, p.h, p.tol, arrival=0.0) for p in probs]
        res = serve_stream(srv, reqs)
    finally:
        srv.close()
    assert len(res) == len(probs)
    for r in res:
        assert r.stats["status"] == bhx.OK, r.stats
    torch.cuda.synchronize()
    for p, q in zip(probs, reqs):
        s, st, ref_alone = alone(handle, p)
        assert s == bhx.OK
        assert np.array_equal(q.F.cpu().numpy(), ref_alone)


def test_requests_join_running_batch(handle):
    """Later arrivals are admitted while earlier requests iterate; every
    result still equals the request solved alone."""
    probs = mixed_requests(8, seed=11, nmin=60, nmax=200, tol=1e-10)
    srv = Server(0, hbm_budget=1 << 30, max_slots=8, chunk=4)
    try:
        reqs = [Request(dev(p.phi), dev(p.F), p.bc, p.h, p.tol, arrival=0.004 * i)
                for i, p in enumerate(probs)]
        res = serve_stream(srv, reqs)
    finally:
        srv.close()
    assert len(res) == len(probs)
    # at least one request was submitted before an earlier one completed
    overlap = any(a.t_submit < b.t_done and a is not b for a in res for b in res
                  if b.request.arrival < a.request.arrival)
    assert overlap
    for p, q in zip(probs, reqs):
        _, _, ref_alone = alone(handle, p)
        assert np.array_equal(q.F.cpu().numpy(), ref_alone)


def test_admission_by_slots_and_budget():
    p = W.circle_problem(64, tol=1e-10)
    srv = Server(0, hbm_budget=64 << 20, max_slots=2)
    try:
        phi = dev(p.phi)
        Fs = [dev(p.F) for _ in range(3)]
        ids = [srv.submit(Request(phi, F, p.bc, p.h, p.tol)) for F in Fs]
        # two slots: the third is refused now (unless the first already finished)
        assert ids[0] is not None and ids[1] is not None
        done = 0
        t0 = time.time()
        while done < 2 and time.time() - t0 < 30:
            done += len(srv.poll())
            time.sleep(1e-3)
        assert done == 2
        assert srv.submit(Request(phi, Fs[2], p.bc, p.h, p.tol)) is not None
        # a request larger than the whole budget can never be admitted
        big = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda:0")
        s, _ = bhx.engine_submit(srv.engine, big, big.clone(), 2048, 2048, 1.0, 0, 1e-8)
        assert s == bhx.ERR_ARG
        t0 = time.time()
        while srv.inflight() and time.time() - t0 < 30:
            srv.poll()
            time.sleep(1e-3)
    finally:
        srv.close()


def test_error_statuses_per_request():
    n = 32
    F = np.random.default_rng(0).normal(size=(n, n))
    srv = Server(0, hbm_budget=256 << 20, max_slots=4)
    try:
        reqs = [Request(dev(np.ones((n, n))), dev(F), 0, 1.0, 1e-8),        # nothing known
                Request(dev(-np.ones((n, n))), dev(F), 0, 1.0, 1e-8),       # nothing unknown
                Request(dev(W.circle_problem(n).phi), dev(W.circle_problem(n).F), 0, 1.0, 1e-10)]
        res = {id(r.request): r for r in serve_stream(srv, reqs)}
    finally:
        srv.close()
    assert res[id(reqs[0])].stats["status"] == bhx.ERR_SINGULAR
    assert np.array_equal(reqs[0].F.cpu().numpy(), F)
    assert res[id(reqs[1])].stats["status"] == bhx.OK
    assert res[id(reqs[1])].stats["iterations"] == 0
    assert res[id(reqs[2])].stats["status"] == bhx.OK
