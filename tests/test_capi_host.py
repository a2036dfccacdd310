"""Host-side checks of the C interface: the library loads, exports every
function include/bhx.h declares, and rejects bad arguments before touching a
GPU.  No compute call is made here."""
import ctypes
import os

import pytest

from paper_1704_08897_amd import bhx


def test_exports_every_declared_symbol():
    names = bhx.header_functions()
    assert "bhx_extend" in names and "bhx_extend_batched" in names
    assert "bhx_engine_submit" in names and "bhx_workspace_bytes" in names
    missing = [n for n in names if not bhx.exported(n)]
    assert not missing, missing


def test_one_hip_runtime_in_process():
    """torch bundles a HIP runtime; importing the binding must not add a
    second one (two runtimes in one process cannot both reach the GPU)."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                paths.add(os.path.realpath(parts[-1]))
    assert len(paths) <= 1, sorted(paths)


def test_default_opts_and_strings():
    o = bhx.default_opts()
    assert (o.precision, o.maxit, o.precond, o.accurate, o.flexible, o.chunk) == (0, 0, 1, 0, -1, 0)
    assert o.warm_start == 0               # x0 = 0 unless asked
    assert bhx.status_string(bhx.OK) == "ok"
    assert "singular" in bhx.status_string(bhx.ERR_SINGULAR)
    assert bhx.status_string(12345) == "unknown status"
    assert "gfx950" in bhx.version()


FAKE = 0x1000  # never dereferenced: validation fails first


@pytest.mark.parametrize("nx,ny,h,bc,tol", [
    (3, 8, 1.0, 0, 1e-8),            # too small
    (8, 2, 1.0, 0, 1e-8),
    (8, 8, 0.0, 0, 1e-8),            # h <= 0
    (8, 8, float("nan"), 0, 1e-8),
    (8, 8, 1.0, 0, 0.0),             # tol outside (0, 1)
    (8, 8, 1.0, 0, 1.0),
    (8, 8, 1.0, 0, float("inf")),
    (8, 8, 1.0, 3, 1e-8),            # bad bc nibble
    (8, 8, 1.0, 0x300, 1e-8),
    (8, 8, 1.0, -1, 1e-8),
    (5000, 8, 1.0, 0, 1e-8),         # transform length not supported
])
def test_extend_rejects_bad_arguments(nx, ny, h, bc, tol):
    assert bhx._lib.bhx_extend(FAKE, FAKE, nx, ny, h, bc, tol) == bhx.ERR_ARG


def test_null_pointers_and_handles():
    assert bhx._lib.bhx_extend(None, FAKE, 8, 8, 1.0, 0, 1e-8) == bhx.ERR_ARG
    assert bhx._lib.bhx_extend(FAKE, None, 8, 8, 1.0, 0, 1e-8) == bhx.ERR_ARG
    s, _ = bhx.extend_ex(None, FAKE, FAKE, 8, 8, 1.0, 0, 1e-8)
    assert s == bhx.ERR_ARG
    assert bhx._lib.bhx_create(None, 0) == bhx.ERR_ARG
    st = (bhx.Stats * 1)()
    assert bhx._lib.bhx_extend_batched(None, 1, None, None, None, None, None, None, None, None,
                                       None, st) == bhx.ERR_ARG
    s, _ = bhx.extend_fields(None, FAKE, [FAKE], nx=8, ny=8)
    assert s == bhx.ERR_ARG
    s, _ = bhx.extend_fields(FAKE, FAKE, [], nx=8, ny=8)          # no field
    assert s == bhx.ERR_ARG
    s, _ = bhx.extend_fields(FAKE, None, [FAKE], nx=8, ny=8)      # no phi
    assert s == bhx.ERR_ARG
    s, _ = bhx.extend_fields(FAKE, FAKE, [FAKE, FAKE + 64, FAKE], nx=8, ny=8)   # one F twice
    assert s == bhx.ERR_ARG
    s, _ = bhx.extend_fields(FAKE, FAKE, [FAKE], nx=3, ny=8)      # bad size
    assert s == bhx.ERR_ARG


def test_bad_options_rejected():
    for kw in ({"precision": 2}, {"precond": 3}, {"maxit": -1}, {"flexible": 2},
               {"tol_inner": 2.0}, {"accurate": 5}, {"warm_start": 2}, {"warm_start": -1},
               {"transform": 3}, {"transform": -1}):
        o = bhx.default_opts(**kw)
        s, _ = bhx.extend_ex(FAKE, FAKE, FAKE, 8, 8, 1.0, 0, 1e-8, opts=o)
        assert s == bhx.ERR_ARG, kw
    assert bhx.workspace_bytes(64, 64, 0, bhx.default_opts(precision=7)) == 0


def test_workspace_bytes():
    w64 = bhx.workspace_bytes(1024, 1024, 0)
    w32 = bhx.workspace_bytes(1024, 1024, 0, bhx.default_opts(precision=1))
    N = 1024 * 1024
    # mask + five float64 vectors + transform buffer (+ small tails)
    assert 49 * N <= w64 < 49 * N + 2 * 1024 * 1024
    assert 45 * N <= w32 < 45 * N + 2 * 1024 * 1024
    assert bhx.workspace_bytes(3, 64, 0) == 0
    assert bhx.workspace_bytes(100, 77, bhx.BC(1, 0)) > 0
    # Dirichlet axes: DST-I through an FFT of the odd extension, length 2(n+1)
    assert bhx.workspace_bytes(64, 64, bhx.BC(2, 0)) > 0
    assert bhx.workspace_bytes(1023, 1023, bhx.BC(2, 2)) > 0          # core length 2048
    assert bhx.workspace_bytes(1000, 64, bhx.BC(2, 0)) > 0            # Bluestein core 4096
    # 1024-2046 nodes: a chirp-z DST-I of n + 1 points, Bluestein core 4096
    for n in (1024, 1100, 1500, 2046):
        assert bhx.workspace_bytes(n, n, bhx.BC(2, 2)) > 0
        assert bhx.workspace_bytes(n, 64, bhx.BC(0, 2), bhx.default_opts(precision=1)) > 0
    assert bhx.workspace_bytes(2047, 64, bhx.BC(2, 0)) > 0            # odd extension, core 4096
    assert bhx.workspace_bytes(2048, 64, bhx.BC(2, 0)) == 0           # core 8192: too long
    assert bhx.workspace_bytes(64, 64, bhx.BC(3, 0)) == 0             # no such rule


def test_engine_rejects_without_device():
    e = ctypes.c_void_p()
    assert bhx._lib.bhx_engine_create(ctypes.byref(e), -1, 1 << 30, 4, None) == bhx.ERR_ARG


def test_three_dimensional_arguments():
    """bhx_extend3d / bhx_workspace_bytes3d / bhx_debug_apply3d reject bad
    arguments on the host."""
    n3 = 64 ** 3
    w = bhx.workspace_bytes3d(64, 64, 64, bhx.BC3(1, 1, 1))
    # mask + five float64 vectors + transform buffer (+ small tails)
    assert 49 * n3 <= w < 49 * n3 + 2 * 1024 * 1024
    assert bhx.workspace_bytes3d(64, 64, 3, 0) == 0                  # nz < 4
    assert bhx.workspace_bytes3d(64, 64, 64, 0x300) == 0             # no such z rule
    assert bhx.workspace_bytes3d(64, 64, 64, 0x1000) == 0            # bits beyond z
    assert bhx.workspace_bytes3d(1024, 1024, 2048, 0) == 0           # 2^31 nodes
    assert bhx.workspace_bytes3d(100, 75, 33, bhx.BC3(2, 1, 0)) > 0  # Bluestein, Dirichlet
    assert bhx.workspace_bytes3d(64, 64, 1100, bhx.BC3(0, 0, 2)) == 0   # no chirp-z along z
    assert bhx.workspace_bytes3d(64, 1100, 64, bhx.BC3(0, 2, 0)) == 0   # nor along y
    s, _ = bhx.extend3d(None, FAKE, FAKE, 8, 8, 8)
    assert s == bhx.ERR_ARG
    for args in [(8, 8, 3, 0), (8, 8, 8, 0x300), (3, 8, 8, 0), (8, 8, 8, -1)]:
        nx, ny, nz, bc = args
        s, _ = bhx.extend3d(FAKE, FAKE, FAKE, nx, ny, nz, bc=bc)
        assert s == bhx.ERR_ARG, args
    s, _ = bhx.extend3d(FAKE, FAKE, FAKE, 8, 8, 8, tol=2.0)
    assert s == bhx.ERR_ARG
    assert bhx.debug_apply3d(FAKE, 2, FAKE, FAKE, FAKE, 8, 8, 8) == bhx.ERR_ARG
    assert bhx.debug_apply3d(FAKE, 0, FAKE, FAKE, FAKE, 8, 8, 2) == bhx.ERR_ARG


def test_direct_solver_option_checks():
    """solver = 1 (banded Cholesky): FP64, at most one periodic axis, two
    dimensions, not the engine; anything else is rejected on the host."""
    assert bhx.default_opts().solver == 0
    for kw, bc in (({"solver": 2}, 0), ({"solver": 1}, bhx.BC(1, 1)),
                   ({"solver": 1, "precision": 1}, 0)):
        s, _ = bhx.extend_ex(FAKE, FAKE, FAKE, 8, 8, 1.0, bc, 1e-8, opts=bhx.default_opts(**kw))
        assert s == bhx.ERR_ARG, kw
    s, _ = bhx.extend3d(FAKE, FAKE, FAKE, 8, 8, 8, opts=bhx.default_opts(solver=1))
    assert s == bhx.ERR_ARG
    e = ctypes.c_void_p()
    assert bhx._lib.bhx_engine_create(ctypes.byref(e), 0, 1 << 30, 4,
                                      ctypes.byref(bhx.default_opts(solver=1))) == bhx.ERR_ARG
