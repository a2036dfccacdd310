"""The allocation-free entry point (bhx_extend_noalloc) against bhx_extend_ex
through the C interface: two calls in a row, the second on a smaller input,
each bit-identical to bhx_extend_ex with the same options (same kernels in
the same order; only where the buffers live differs) and within the FP64
bar of the oracle; inputs too large for the scratch array are refused with
F untouched."""
import numpy as np
import pytest

import oracle as O
from paper_1704_08897_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08897_amd import bhx  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def star(nx, ny, bx, by, seed):
    rng = np.random.default_rng(seed)
    h = 2.0 / min(nx, ny)
    X, Y = np.meshgrid(W.axis_nodes(nx, -nx * h / 2, nx * h / 2, bx),
                       W.axis_nodes(ny, -ny * h / 2, ny * h / 2, by))
    th = np.arctan2(Y, X)
    r = 0.55 * (1 + 0.1 * np.cos(5 * th + rng.uniform(0, 6)))
    phi = np.hypot(X, Y) - r
    F = np.sin(1.3 * X) * np.cos(Y) + 0.2 * X * Y
    return W.Problem(phi, F, bx, by, h, 1e-12)


@pytest.fixture(scope="module")
def handle():
    h = bhx.Handle(0)
    yield h
    h.close()


def test_noalloc_matches_extend_ex_twice(handle):
    # the first call larger (Neumann x periodic, Bluestein on x), the second
    # smaller (Dirichlet x Neumann): the second must not see the first's state
    cases = [star(600, 512, 0, 1, 1), star(130, 97, 2, 0, 2)]
    for p in cases:
        o = bhx.default_opts()
        phi = dev(p.phi)
        Fa = dev(p.F)
        Fb = dev(p.F)
        sa, sta = bhx.extend_noalloc(handle, phi, Fa, bc=p.bc, h=p.h, tol=p.tol, opts=o)
        sb, stb = bhx.extend_ex(handle, phi, Fb, bc=p.bc, h=p.h, tol=p.tol, opts=o)
        assert sa == bhx.OK and sb == bhx.OK, (bhx.status_string(sa), bhx.last_error())
        assert sta.iterations == stb.iterations and sta.n_unknown == stb.n_unknown
        assert sta.true_rel_residual <= p.tol
        torch.cuda.synchronize()
        a, b = Fa.cpu().numpy(), Fb.cpu().numpy()
        assert np.array_equal(a, b)
        ref, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
        assert np.array_equal(a[p.phi < 0], p.F[p.phi < 0])
        assert O.relative_l2(a, ref) <= 1e-9


def test_noalloc_options_and_limits(handle):
    # accurate mode and the FP32 preconditioner run on the scratch too
    p = star(200, 180, 1, 1, 3)
    for kw in ({"accurate": 1, "tol_inner": 1e-8}, {"precision": 1}):
        o = bhx.default_opts(**kw)
        Fa, Fb = dev(p.F), dev(p.F)
        sa, sta = bhx.extend_noalloc(handle, dev(p.phi), Fa, bc=p.bc, h=p.h, tol=1e-12, opts=o)
        sb, stb = bhx.extend_ex(handle, dev(p.phi), Fb, bc=p.bc, h=p.h, tol=1e-12, opts=o)
        assert sa == sb == bhx.OK
        assert torch.equal(Fa, Fb)
    # too large for the scratch array: refused, F untouched, the reason given
    big = W.circle_problem(1600, tol=1e-8)
    F = dev(big.F)
    s, _ = bhx.extend_noalloc(handle, dev(big.phi), F, bc=big.bc, h=big.h, tol=big.tol)
    assert s == bhx.ERR_ARG
    assert "limit" in bhx.last_error()
    assert torch.equal(F, dev(big.F))
    # options it does not take
    s, _ = bhx.extend_noalloc(handle, dev(p.phi), dev(p.F), bc=p.bc, h=p.h, tol=1e-8,
                              opts=bhx.default_opts(autotune=1))
    assert s == bhx.ERR_ARG
