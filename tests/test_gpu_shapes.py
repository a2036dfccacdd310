"""GPU parity of the compile-time-shape transform kernels: an instance (or a
batch of same-shape instances) whose x or y axis has 64 to 2048 nodes (a
power of two) with the Neumann or periodic rule, or 63 to 2047 nodes (n + 1 a
power of two) with the Dirichlet rule, runs instances of the row and column passes with that shape
fixed at compile time.  Checked against the oracle's spectral preconditioner and sparse
direct extension, and against the same launches with the shape kernels
switched off (BHX_SHAPE_KERNELS=0, read at every call).

Bounds: the preconditioner within relative L2 1e-11 of the oracle, as in the
generic parity tests; the two kernel families perform the same operations in
the same order (only constant folding and contraction differ), so their
preconditioner outputs agree within 1e-13.  Solved fields at tol 1e-12 within
1e-9 of the oracle (the star's conditioning, as in the full-size tests).
Every call here asks for the FFT family (bhx_opts.transform = 1): the
built-in choice would run some of these sizes as dense products."""
import numpy as np
import pytest

import oracle as O
from paper_1704_08897_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1704_08897_amd import bhx  # noqa: E402

DEV = "cuda:0"
FFT = bhx.default_opts(transform=1)


@pytest.fixture(scope="module")
def handle():
    h = bhx.Handle(0)
    yield h
    h.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def apply_precond(handle, phi, r, bx, by):
    out = dev(np.zeros_like(r))
    assert bhx.debug_apply(handle, 1, dev(phi), dev(r), out, bc=bhx.BC(bx, by),
                           transform=1) == bhx.OK
    return host(out)


# (nx, ny, bcx, bcy): both axes shaped; one shaped and one generic (Bluestein
# length, Dirichlet rule on a non-shaped length); a length just outside the
# instantiated set; ragged last groups on a shaped axis (an odd row count under
# the x shape, an odd column count under the y shape); Dirichlet axes of 63 to
# 2047 nodes (DST-I through 128- to 4096-point cores)
CASES = [(512, 512, 0, 0), (1024, 512, 1, 0), (512, 2048, 0, 1), (2048, 1024, 1, 1),
         (1024, 1000, 0, 0), (1000, 1024, 1, 0), (1024, 1023, 0, 2), (256, 1024, 0, 1),
         (1024, 333, 1, 0), (257, 1024, 0, 1), (2048, 77, 0, 0),
         (1023, 511, 2, 2), (1023, 1024, 2, 0), (511, 1023, 1, 2), (1023, 100, 2, 1),
         (255, 127, 2, 2), (63, 255, 2, 0), (2047, 64, 2, 1)]


@pytest.mark.parametrize("nx,ny,bx,by", CASES)
def test_preconditioner_shapes(handle, monkeypatch, nx, ny, bx, by):
    rng = np.random.default_rng(nx + 3 * ny + bx + by)
    phi = -(rng.random((ny, nx)) - 0.3)
    r = rng.normal(size=(ny, nx))
    known = O.known_mask(phi)
    ref = O.spectral_preconditioner(r, known, bx, by)
    got = apply_precond(handle, phi, r, bx, by)
    assert np.array_equal(got[known], np.zeros(known.sum()))
    assert O.relative_l2(got, ref) <= 1e-11
    monkeypatch.setenv("BHX_SHAPE_KERNELS", "0")
    generic = apply_precond(handle, phi, r, bx, by)
    assert O.relative_l2(got, generic) <= 1e-13


def test_star1024_solve_shapes(handle, monkeypatch):
    """The benchmark star through the shape kernels (both axes 1024, Neumann)
    and through the generic ones: both meet the tolerance and the oracle."""
    p = W.star_inward_problem(1024, tol=1e-12)
    Fo, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
    K = O.known_mask(p.phi)
    res = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BHX_SHAPE_KERNELS", flag)
        G = dev(p.F)
        s, st = bhx.extend_ex(handle, dev(p.phi), G, bc=p.bc, h=p.h, tol=p.tol, opts=FFT)
        assert s == bhx.OK, st.as_dict()
        got = host(G)
        assert np.array_equal(got[K], p.F[K])
        assert O.true_relative_residual(K, p.F, got, p.bcx, p.bcy) <= p.tol * 1.001
        assert O.relative_l2(got, Fo) <= 1e-9
        res[flag] = (got, st.iterations)
    # same Krylov method on operators equal to rounding: iteration counts close
    assert abs(res["1"][1] - res["0"][1]) <= 0.05 * res["0"][1]


@pytest.mark.parametrize("make", [lambda: W.peanut_problem(512, 1, 0, tol=1e-12),
                                  lambda: W.annulus_problem(512, 0, 1, tol=1e-12)],
                         ids=["peanut512_periodic_neumann", "annulus512_neumann_periodic"])
def test_paper_masks_solve_shapes(handle, make):
    """Examples 1 and 3's masks on shaped axes of both rules, against the
    oracle's sparse direct extension."""
    p = make()
    Fo, _ = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
    K = O.known_mask(p.phi)
    G = dev(p.F)
    s, st = bhx.extend_ex(handle, dev(p.phi), G, bc=p.bc, h=p.h, tol=p.tol, opts=FFT)
    assert s == bhx.OK, st.as_dict()
    got = host(G)
    assert np.array_equal(got[K], p.F[K])
    assert O.true_relative_residual(K, p.F, got, p.bcx, p.bcy) <= p.tol * 1.001
    assert O.relative_l2(got, Fo) <= 1e-9


def test_fields_and_same_shape_batch(handle):
    """Several fields on one phi, and a batch of two instances of one shape
    (512 x 512, periodic x Neumann), run the shape kernels as a batch: each
    result equals its own one-instance solve bit for bit (per-instance
    reductions in a fixed order) and meets the oracle."""
    p = W.peanut_problem(512, 1, 0, tol=1e-10)
    ny, nx = p.F.shape
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
    fields = [p.F, np.where(O.known_mask(p.phi), X**3 - Y, 0.0)]
    Fs = [dev(f) for f in fields]
    s, sts = bhx.extend_fields(handle, dev(p.phi), Fs, h=p.h, bc=p.bc, tol=p.tol, opts=FFT)
    assert s == bhx.OK
    for f, G in zip(fields, Fs):
        A = dev(f)
        s1, _ = bhx.extend_ex(handle, dev(p.phi), A, bc=p.bc, h=p.h, tol=p.tol, opts=FFT)
        assert s1 == bhx.OK
        assert np.array_equal(host(G), host(A))
    q = W.annulus_problem(512, 1, 0, tol=1e-10)
    batch = [p, q]
    Bs = [dev(b.F) for b in batch]
    s, sts = bhx.extend_batched(handle, [dev(b.phi) for b in batch], Bs, [b.h for b in batch],
                                [b.bc for b in batch], [b.tol for b in batch], opts=FFT)
    assert s == bhx.OK
    for b, G in zip(batch, Bs):
        A = dev(b.F)
        s1, _ = bhx.extend_ex(handle, dev(b.phi), A, bc=b.bc, h=b.h, tol=b.tol, opts=FFT)
        assert s1 == bhx.OK
        got = host(G)
        assert np.array_equal(got, host(A))
        K = O.known_mask(b.phi)
        assert O.true_relative_residual(K, b.F, got, b.bcx, b.bcy) <= b.tol * 1.001


def test_mixed_batch_runs_plan_table_family(handle):
    """A shaped instance (512 x 512, periodic x Neumann) batched with a
    differently shaped one runs the plan-table kernels: it meets the residual
    bar and agrees with its solo (shape-kernel) solve to the solves' accuracy,
    not bit for bit (a batch of equal shapes does reproduce the solo solve bit
    for bit, test_fields_and_same_shape_batch)."""
    p = W.peanut_problem(512, 1, 0, tol=1e-12)
    q = W.circle_problem(64, tol=1e-12)
    Bs = [dev(p.F), dev(q.F)]
    s, sts = bhx.extend_batched(handle, [dev(p.phi), dev(q.phi)], Bs, [p.h, q.h], [p.bc, q.bc],
                                [p.tol, q.tol], opts=FFT)
    assert s == bhx.OK
    got = host(Bs[0])
    A = dev(p.F)
    s1, _ = bhx.extend_ex(handle, dev(p.phi), A, bc=p.bc, h=p.h, tol=p.tol, opts=FFT)
    assert s1 == bhx.OK
    solo = host(A)
    K = O.known_mask(p.phi)
    assert np.array_equal(got[K], p.F[K])
    assert O.true_relative_residual(K, p.F, got, p.bcx, p.bcy) <= p.tol * 1.001
    assert O.relative_l2(got, solo) <= 1e-9


@pytest.mark.parametrize("nx,ny,bx,by", [(1024, 512, 0, 1), (2048, 333, 1, 0), (1023, 511, 2, 2)])
def test_preconditioner_shapes_fp32(handle, monkeypatch, nx, ny, bx, by):
    """FP32 transforms through the shape instances: within the FP32 bound of
    the generic tests (2e-4) of the oracle, and within 1e-5 of the plan-table
    FP32 kernels (the same operations; contraction differs, at FP32
    rounding amplified by the 1/Lambda^2 spread)."""
    rng = np.random.default_rng(nx + ny)
    phi = -(rng.random((ny, nx)) - 0.3)
    r = rng.normal(size=(ny, nx))
    known = O.known_mask(phi)
    ref = O.spectral_preconditioner(r, known, bx, by)
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BHX_SHAPE_KERNELS", flag)
        out = dev(np.zeros_like(r))
        assert bhx.debug_apply(handle, 1, dev(phi), dev(r), out, bc=bhx.BC(bx, by),
                               precision=1, transform=1) == bhx.OK
        outs.append(host(out))
    assert np.array_equal(outs[0][known], np.zeros(known.sum()))
    assert O.relative_l2(outs[0], ref) <= 2e-4
    assert O.relative_l2(outs[0], outs[1]) <= 1e-5


def test_star1024_fp32_solve_shapes(handle, monkeypatch):
    """The star with the FP32 preconditioner (standard PCG) through both
    kernel families: both meet tol 1e-8 with the true residual.  Iteration
    counts within 15 %: FP32 rounding of the preconditioner (about 1e-7
    relative, amplified by the 1/Lambda^2 spread) moves the Krylov path far
    more than FP64 rounding does (measured 3,823 against 4,098)."""
    p = W.star_inward_problem(1024, tol=1e-8)
    K = O.known_mask(p.phi)
    its = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BHX_SHAPE_KERNELS", flag)
        G = dev(p.F)
        s, st = bhx.extend_ex(handle, dev(p.phi), G, bc=p.bc, h=p.h, tol=p.tol,
                              opts=bhx.default_opts(precision=1, transform=1))
        assert s == bhx.OK, st.as_dict()
        got = host(G)
        assert np.array_equal(got[K], p.F[K])
        assert O.true_relative_residual(K, p.F, got, p.bcx, p.bcy) <= p.tol * 1.001
        its.append(st.iterations)
    assert abs(its[0] - its[1]) <= 0.15 * its[1]


def test_dirichlet_star1023_solve_shapes(handle, monkeypatch):
    """The star on 1023 x 1023 with Dirichlet rules on both axes (shape
    instances with the DST-I through 2048-point cores) and through the
    plan-table kernels: both meet tol with the true residual and agree with
    the oracle's sparse direct extension within 1e-9 at tol 1e-12."""
    s0 = W.star_inward_problem(1023, tol=1e-12)
    bc = bhx.BC(2, 2)
    Fo, _ = O.extend_direct(s0.phi, s0.F, 2, 2)
    K = O.known_mask(s0.phi)
    its = []
    for flag in ("1", "0"):
        monkeypatch.setenv("BHX_SHAPE_KERNELS", flag)
        G = dev(s0.F)
        s, st = bhx.extend_ex(handle, dev(s0.phi), G, bc=bc, h=s0.h, tol=1e-12, opts=FFT)
        assert s == bhx.OK, st.as_dict()
        got = host(G)
        assert np.array_equal(got[K], s0.F[K])
        assert O.true_relative_residual(K, s0.F, got, 2, 2) <= 1e-12 * 1.001
        assert O.relative_l2(got, Fo) <= 1e-9
        its.append(st.iterations)
    assert abs(its[0] - its[1]) <= 0.05 * its[1]
