"""GPU parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (default options unless stated).

Where the CPU oracle can solve the case in test time (the 1024 x 1024 star,
batch instances, serving requests up to ~1200 x 1200) the result is compared
with it.  The 2048 x 2048 periodic case (2.2 M unknowns, about ten minutes of
SuperLU) is compared with the oracle's solution at sampled nodes, stored by
tests/golden/make_periodic_2048_sample.py.  At every size, properties that
hold at any size are checked too:
- the relative residual of the returned field, recomputed on the CPU in long
  double from the inputs, meets the tolerance;
- known values are returned bit for bit.

Error bounds.  At tol 1e-8 the error is bounded only by the condition number
(~1e9-1e11 here) times the residual, so the asserted bounds at that tol are
empirical: observed values with a stated margin.  The tight bars (1e-9 for
FP64) are asserted where the solve is run to a tolerance that supports them:
accurate mode at tol 1e-13, or plain PCG at tol 1e-12.
"""
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


@pytest.fixture(scope="module")
def handle():
    h = bhx.Handle(0)
    yield h
    h.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def solve(handle, p, tol=None, **opts):
    F = dev(p.F)
    s, st = bhx.extend_ex(handle, dev(p.phi), F, bc=p.bc, h=p.h, tol=tol or p.tol,
                          opts=bhx.default_opts(**opts))
    torch.cuda.synchronize()
    return s, st, F.cpu().numpy()


def check_properties(p, got, tol):
    known = O.known_mask(p.phi)
    assert np.array_equal(got[known], p.F[known])
    res = O.true_relative_residual(known, p.F, got, p.bcx, p.bcy)
    assert res <= tol * 1.001, res
    return res


@pytest.fixture(scope="module")
def star1024():
    p = W.star_inward_problem(1024, tol=1e-8)
    ref, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
    return p, ref


def test_star1024_bench_configuration(handle, star1024):
    """Configuration of the default benchmark: FP64 PCG, tol 1e-8."""
    p, ref = star1024
    s, st, got = solve(handle, p)
    assert s == bhx.OK
    assert 900 <= st.iterations <= 980
    res = check_properties(p, got, 1e-8)
    assert abs(res - st.true_rel_residual) <= 1e-3 * res      # GPU's own true residual agrees
    err = O.relative_l2(got, ref)
    assert err <= 3e-6, err           # observed 3.3e-7; margin 10x


def test_star1024_accurate_mode_meets_fp64_bar(handle, star1024):
    """Accurate mode (defect correction) at tol 1e-13: the FP64 bar 1e-9."""
    p, ref = star1024
    s, st, got = solve(handle, p, tol=1e-13, accurate=1, tol_inner=1e-8)
    assert s == bhx.OK
    check_properties(p, got, 1e-13)
    assert O.relative_l2(got, ref) <= 1e-9


def test_star1024_fp32_preconditioner(handle, star1024):
    """FP32 transforms, FP64 recurrences, tol 1e-12: the mixed bar 1e-8."""
    p, ref = star1024
    s, st, got = solve(handle, p, tol=1e-12, precision=1)
    assert s == bhx.OK
    check_properties(p, got, 1e-12)
    assert O.relative_l2(got, ref) <= 1e-8


def test_periodic2048_properties(handle):
    """2048 x 2048 periodic, 20 circles, FP64, tol 1e-8 (too large for the
    direct oracle in test time): residual recomputed in long double on the
    CPU, known values untouched."""
    p = W.periodic_circles_problem(2048, tol=1e-8)
    s, st, got = solve(handle, p)
    assert s == bhx.OK
    res = check_properties(p, got, 1e-8)
    assert abs(res - st.true_rel_residual) <= 1e-3 * res


def test_batch256_sampled_instances(handle):
    """The 256-instance batch as the benchmark runs it (FP64, autotuned,
    tol 1e-8): every instance meets the tolerance by the CPU residual."""
    batch = W.star_cubic_batch(256, seed=4, tol=1e-8)
    phis = [dev(p.phi) for p in batch]
    Fs = [dev(p.F) for p in batch]
    s, sts = bhx.extend_batched(handle, phis, Fs, [p.h for p in batch], [p.bc for p in batch],
                                [p.tol for p in batch], opts=bhx.default_opts(autotune=1))
    assert s == bhx.OK
    torch.cuda.synchronize()
    for i in range(0, 256, 16):
        check_properties(batch[i], Fs[i].cpu().numpy(), 1e-8)


# instances of the 256-instance batch compared with the oracle: both known
# sides, both rules on each axis, sides from 70 to 500
BATCH_SAMPLE = [3, 17, 40, 74, 101, 152, 188, 220, 241, 255]


@pytest.fixture(scope="module")
def batch_sample_refs():
    batch = W.star_cubic_batch(256, seed=4, tol=1e-8)
    probs = [batch[i] for i in BATCH_SAMPLE]
    refs = [O.extend_direct(p.phi, p.F, p.bcx, p.bcy)[0] for p in probs]
    return probs, refs


@pytest.mark.parametrize("prec,bar", [(0, 1e-9), (1, 1e-8)])
def test_batch256_sample_accurate_mode_meets_bar(handle, batch_sample_refs, prec, bar):
    """Instances of the batch solved together in one batched call in accurate
    mode (defect correction with the compensated residual, tol 1e-13): each
    meets the stated bar against the oracle, 1e-9 with the FP64
    preconditioner and 1e-8 with the FP32 one.  At the batch's own tol 1e-8
    the error is bounded only by the condition number times the residual
    (observed up to a few 1e-5), which is why the bar is asserted here."""
    probs, refs = batch_sample_refs
    Fs = [dev(p.F) for p in probs]
    o = bhx.default_opts(precision=prec, accurate=1, tol_inner=1e-8)
    s, sts = bhx.extend_batched(handle, [dev(p.phi) for p in probs], Fs, [p.h for p in probs],
                                [p.bc for p in probs], [1e-13] * len(probs), opts=o)
    assert s == bhx.OK, [st.as_dict() for st in sts]
    torch.cuda.synchronize()
    errs = []
    for p, F, ref, st in zip(probs, Fs, refs, sts):
        got = F.cpu().numpy()
        check_properties(p, got, 1e-13)
        errs.append(O.relative_l2(got, ref))
    assert max(errs) <= bar, errs


def serving_sample():
    """Requests of the serving mix: the first ones of side <= 520 and the
    first one of side in (1024, 1200], drawn in stream order (seed 5)."""
    specs = W.request_stream(400, seed=5)
    small = [s for s in specs if s.n <= 520][:5]
    large = [s for s in specs if 1024 < s.n <= 1200][:1]
    assert len(large) == 1
    return [s.materialise() for s in small + large]


def test_serving_mix_properties():
    """Requests of the serving mix through the engine together at tol 1e-8
    (the configuration the benchmark serves): each meets the tolerance by
    the CPU residual, known values bit for bit."""
    specs = W.request_stream(400, seed=5)
    probs = [s.materialise() for s in [s for s in specs if s.n <= 520][:6] +
             [s for s in specs if 900 <= s.n <= 1400][:2]]
    srv = Server(0, hbm_budget=8 << 30, max_slots=16)
    try:
        reqs = [Request(dev(p.phi), dev(p.F), p.bc, p.h, p.tol, arrival=0.0) for p in probs]
        res = serve_stream(srv, reqs)
    finally:
        srv.close()
    assert len(res) == len(probs)
    assert all(r.stats["status"] == bhx.OK for r in res)
    torch.cuda.synchronize()
    for p, q in zip(probs, reqs):
        check_properties(p, q.F.cpu().numpy(), p.tol)


def test_serving_mix_accurate_mode_meets_fp64_bar():
    """The engine in accurate mode (tol 1e-13): a mix of serving requests,
    one of side above 1024, each within 1e-9 of the oracle.  At the mix's
    own tol 1e-8 only the residual is bounded (previous test)."""
    probs = serving_sample()
    refs = [O.extend_direct(p.phi, p.F, p.bcx, p.bcy)[0] for p in probs]
    srv = Server(0, hbm_budget=8 << 30, max_slots=16, accurate=1, tol_inner=1e-8)
    try:
        reqs = [Request(dev(p.phi), dev(p.F), p.bc, p.h, 1e-13, arrival=0.0) for p in probs]
        res = serve_stream(srv, reqs)
    finally:
        srv.close()
    assert len(res) == len(probs)
    assert all(r.stats["status"] == bhx.OK for r in res), [r.stats for r in res]
    torch.cuda.synchronize()
    errs = []
    for p, q, ref in zip(probs, reqs, refs):
        got = q.F.cpu().numpy()
        check_properties(p, got, 1e-13)
        errs.append((p.nx, O.relative_l2(got, ref)))
    assert max(e for _, e in errs) <= 1e-9, errs


def read_periodic_sample():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "periodic_circles_2048_sample.txt")
    meta, idx, val = {}, [], []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        if "=" in line:
            k, v = line.split("=", 1)
            meta[k.strip()] = v.strip()
        else:
            a, b = line.split()
            idx.append(int(a))
            val.append(float(b))
    return meta, np.array(idx), np.array(val)


@pytest.mark.parametrize("prec,bar", [(1, 1e-8), (0, 1e-9)])
def test_periodic2048_against_stored_oracle_sample(handle, prec, bar):
    """The 2048 x 2048 periodic configuration (20 circles, seed 3) against the
    oracle's solution at ~2,100 sampled unknown nodes, stored by
    tests/golden/make_periodic_2048_sample.py (SuperLU plus long-double
    refinement).  The FP32 preconditioner (the configuration's precision)
    and the FP64 one, each in accurate mode at tol 1e-13: relative L2 over
    the sample within the stated bar, 1e-8 mixed and 1e-9 FP64."""
    meta, idx, val = read_periodic_sample()
    p = W.periodic_circles_problem(2048, seed=int(meta["seed"]), tol=1e-13)
    assert int(meta["nx"]) == p.nx and int(meta["n_unknown"]) == int((p.phi >= 0).sum() +
                                                                      np.isnan(p.phi).sum())
    # the FP32 preconditioner needs about 55k iterations per 1e-8 of reduction
    # here, so two outer steps exceed the default limit (50 x 2048)
    s, st, got = solve(handle, p, tol=1e-13, precision=prec, accurate=1, tol_inner=1e-8,
                       maxit=400000)
    assert s == bhx.OK, st.as_dict()
    assert st.true_rel_residual <= 1e-13
    g = got.ravel()[idx]
    err = np.linalg.norm(g - val) / np.linalg.norm(val)
    assert err <= bar, err
