"""Plain CPU reference for the masked discrete biharmonic extension.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run this module; the
GPU library never does.  It shares no code, table or helper with the HIP
path.

What it computes (Sec. 2.1-2.2 of the paper):

* the field is known at grid nodes where the level-set function is negative
  (the region definitions of Sec. 3 use a strict inequality) and unknown at
  every other node;
* at each unknown node the 13-point discrete biharmonic equation, eq. (12),
  holds; the stencil is the 5-point Laplacian applied twice with two layers of
  ghost nodes per boundary (Algorithm 1), so the full-grid operator is
  A = L^2 with L = I (x) T_x + T_y (x) I;
* values at known nodes enter the right-hand side, so the unknowns solve
  A_UU u = -A_UK f_K, a sparse symmetric positive definite system (Sec. 2.2),
  solved here by a sparse direct factorisation (the paper's direct route,
  Sec. 2.2 and Tables 2/5) followed by iterative refinement with a
  long-double residual.

Readings taken where the paper is silent (each is listed with its reason in
the design notes of the repository):

* Dirichlet ghosts follow Algorithm 1: g[-1] = 0, g[-2] = -f[0].
* Neumann ghosts are half-sample symmetric: g[-1] = f[0], g[-2] = f[1]; this
  is the reflection whose operator is symmetric (the paper calls the system
  SPD in Sec. 2.2) and whose eigenvectors are the DCT-II basis (Sec. 3.1 says
  the Neumann variant uses cosine transforms).
* Periodic ghosts wrap around: g[-1] = f[n-1], g[-2] = f[n-2] (Sec. 3.2, 3.4).
* The spectral preconditioner (Algorithm 1, Sec. 2.2) divides by the square
  of the eigenvalues of L; a zero eigenvalue (Neumann/periodic on both axes)
  gets coefficient 0, i.e. the Moore-Penrose pseudo-inverse.
* Eigenvalues are written 4 sin^2(theta/2), equal to 2(1 - cos theta) of
  Algorithm 1 but without cancellation at small theta.

Arrays are (ny, nx), row-major with x fastest: node (i, j) is a[j, i] and
linear index j*nx + i.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

NEUMANN, PERIODIC, DIRICHLET = 0, 1, 2
_BC_NAMES = {NEUMANN: "neumann", PERIODIC: "periodic", DIRICHLET: "dirichlet"}


class SingularProblem(ValueError):
    """No known node and no Dirichlet axis: the extension is defined only up
    to a constant (the operator has the constant null vector)."""


def known_mask(phi):
    """Known set Omega = {phi < 0}, strict (Sec. 3 region definitions).

    phi == 0 and NaN are unknown.  Returns a boolean array of phi's shape.
    """
    return np.asarray(phi) < 0


# ----------------------------------------------------------------------------
# Operator, assembled two independent ways
# ----------------------------------------------------------------------------

def second_difference_1d(n, bc):
    """1-D operator (T f)_i = 2 f_i - f_{i-1} - f_{i+1} with one ghost rule.

    Algorithm 1's padding implies, for the node next to a boundary:
    Dirichlet g[-1] = 0 (plain tridiag(-1, 2, -1)); Neumann g[-1] = f[0]
    (corner entries become 1); periodic g[-1] = f[n-1] (circulant).
    """
    main = np.full(n, 2.0)
    off = np.full(n - 1, -1.0)
    T = sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="lil")
    if bc == NEUMANN:
        T[0, 0] = 1.0
        T[n - 1, n - 1] = 1.0
    elif bc == PERIODIC:
        T[0, n - 1] = -1.0
        T[n - 1, 0] = -1.0
    elif bc != DIRICHLET:
        raise ValueError(f"bad bc {bc}")
    return T.tocsr()


def laplacian(nx, ny, bcx, bcy):
    """Negative 5-point Laplacian L = I_y (x) T_x + T_y (x) I_x (unscaled).

    Row-major, x fastest: kron(I_ny, T_x) acts along each grid row.
    """
    Tx = second_difference_1d(nx, bcx)
    Ty = second_difference_1d(ny, bcy)
    return (sp.kron(sp.identity(ny), Tx) + sp.kron(Ty, sp.identity(nx))).tocsr()


def biharmonic_matrix(nx, ny, bcx, bcy):
    """Full-grid 13-point biharmonic operator A = L^2 (eq. (12) is L^2 in the
    interior: 20 / -8 / 2 / 1).  Sparse CSR, float64, integer entries."""
    L = laplacian(nx, ny, bcx, bcy)
    return (L @ L).tocsr()


def _pad_axis(a, axis, bc):
    """Add two ghost layers on both ends of ``axis`` by the rule of ``bc``."""
    a = np.moveaxis(a, axis, 0)
    n = a.shape[0]
    out = np.zeros((n + 4,) + a.shape[1:], dtype=a.dtype)
    out[2:n + 2] = a
    if bc == DIRICHLET:        # Algorithm 1: g[-1] = 0, g[-2] = -f[0]
        out[0] = -a[0]
        out[n + 3] = -a[n - 1]
    elif bc == NEUMANN:        # half-sample even reflection
        out[1] = a[0]
        out[0] = a[1]
        out[n + 2] = a[n - 1]
        out[n + 3] = a[n - 2]
    elif bc == PERIODIC:       # wrap-around
        out[1] = a[n - 1]
        out[0] = a[n - 2]
        out[n + 2] = a[0]
        out[n + 3] = a[1]
    else:
        raise ValueError(f"bad bc {bc}")
    return np.moveaxis(out, 0, axis)


def _five_point(P):
    """4 c - (four axis neighbours) on the interior of padded array P."""
    return (4 * P[1:-1, 1:-1] - P[:-2, 1:-1] - P[2:, 1:-1]
            - P[1:-1, :-2] - P[1:-1, 2:])


def stencil_padded(f, bcx, bcy):
    """Left-hand side of eq. (12) at every node, the way Algorithm 1 forms it:
    pad the (ny, nx) array with two ghost layers per side (rows, then
    columns), apply the 5-point Laplacian on the one-layer ring, then again on
    the grid.  Works in the dtype of ``f``."""
    f = np.asarray(f)
    P = _pad_axis(_pad_axis(f, 0, bcy), 1, bcx)
    L1 = _five_point(P)          # (ny + 2, nx + 2): grid plus one ring
    return _five_point(L1)       # (ny, nx)


def stencil_padded_ld(f, bcx, bcy):
    """``stencil_padded`` in numpy long double (x86 80-bit, eps ~ 1.1e-19)."""
    return stencil_padded(np.asarray(f, dtype=np.longdouble), bcx, bcy)


# ----------------------------------------------------------------------------
# The masked system and its direct solution
# ----------------------------------------------------------------------------

def rhs(F, known, bcx, bcy):
    """Right-hand side over the unknown nodes (Algorithm 1's first step):
    b = -(A f_K)|_U with f_K equal to F at known nodes and zero elsewhere.
    Returned as a vector over the unknown nodes in row-major order."""
    f = np.where(known, F, 0.0)
    return -stencil_padded(f, bcx, bcy)[~known]


def reduced_system(known, bcx, bcy):
    """A_UU: rows and columns of A = L^2 at the unknown nodes (CSC)."""
    ny, nx = known.shape
    A = biharmonic_matrix(nx, ny, bcx, bcy)
    U = np.flatnonzero(~known.ravel())
    return A[U][:, U].tocsc()


def extend_direct(phi, F, bcx, bcy, refine=2, known=None):
    """Biharmonic extension by sparse direct factorisation (Sec. 2.2).

    Returns (F_out, info).  F_out equals F bit-exactly at known nodes and the
    solution of A_UU u = b at unknown nodes.  ``refine`` steps of iterative
    refinement use a long-double residual computed with the padded stencil,
    i.e. independently of the factorised matrix.
    """
    F = np.asarray(F, dtype=np.float64)
    if known is None:
        known = known_mask(phi)
    unknown = ~known
    F_out = F.copy()
    info = {"n_unknown": int(unknown.sum()), "refine_residuals": []}
    if not unknown.any():
        return F_out, info
    if not known.any() and DIRICHLET not in (bcx, bcy):
        raise SingularProblem("no known node and no Dirichlet axis")
    b = rhs(F, known, bcx, bcy)
    A_UU = reduced_system(known, bcx, bcy)
    lu = spla.splu(A_UU, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options={"SymmetricMode": True})
    u = np.asarray(lu.solve(b), dtype=np.longdouble)
    f_ld = np.asarray(np.where(known, F, 0.0), dtype=np.longdouble)
    b_norm = float(np.linalg.norm(b))
    for _ in range(refine):
        f_ld[unknown] = u
        r = -stencil_padded(f_ld, bcx, bcy)[unknown]     # b - A_UU u, long double
        info["refine_residuals"].append(
            float(np.sqrt(np.sum(r * r))) / b_norm if b_norm > 0 else 0.0)
        u = u + np.asarray(lu.solve(np.asarray(r, dtype=np.float64)), dtype=np.longdouble)
    F_out[unknown] = np.asarray(u, dtype=np.float64)
    return F_out, info


# ----------------------------------------------------------------------------
# Spectral (fast Poisson) preconditioner, Algorithm 1 and Sec. 2.2
# ----------------------------------------------------------------------------

def eigenvalues_1d(n, bc):
    """Eigenvalues of the 1-D operator T in the order of ``transform_1d``'s
    coefficients, as 4 sin^2(theta/2) (= 2(1 - cos theta), Algorithm 1)."""
    k = np.arange(n, dtype=np.float64)
    if bc == NEUMANN:
        theta = np.pi * k / n
    elif bc == PERIODIC:
        theta = 2 * np.pi * k / n
    elif bc == DIRICHLET:
        theta = np.pi * (k + 1) / (n + 1)
    else:
        raise ValueError(f"bad bc {bc}")
    return 4.0 * np.sin(theta / 2) ** 2


def transform_1d(x, bc, axis, inverse=False):
    """Orthonormal eigenbasis transform of T along ``axis``.

    Neumann: DCT-II (inverse DCT-III); Dirichlet: DST-I (Algorithm 1's sine
    transform, self-inverse when orthonormal); periodic: the discrete Hartley
    transform (Re - Im of the DFT), a real orthonormal self-inverse basis of
    the symmetric circulant T (its eigenvalues are even in k).
    """
    if bc == NEUMANN:
        f = sfft.idct if inverse else sfft.dct
        return f(x, type=2, norm="ortho", axis=axis)
    if bc == DIRICHLET:
        return sfft.dst(x, type=1, norm="ortho", axis=axis)
    if bc == PERIODIC:
        X = sfft.fft(x, axis=axis, norm="ortho")
        return X.real - X.imag
    raise ValueError(f"bad bc {bc}")


def spectral_preconditioner(r, known, bcx, bcy):
    """z = R T^T diag(1/Lambda^2) T R^T r (Algorithm 1's preconditioner).

    ``r`` is a full-grid (ny, nx) array; it is embedded by zeroing the known
    nodes (Sec. 2.2), transformed along x then y, divided by
    (lambda_x + lambda_y)^2 (zero where that vanishes), transformed back and
    restricted (zero at known nodes).  With ``known`` all False this is the
    (pseudo-)inverse of A on the full grid.
    """
    ny, nx = r.shape
    R = np.where(known, 0.0, r)
    X = transform_1d(transform_1d(R, bcx, axis=1), bcy, axis=0)
    lam = eigenvalues_1d(ny, bcy)[:, None] + eigenvalues_1d(nx, bcx)[None, :]
    with np.errstate(divide="ignore"):
        w = np.where(lam > 0, 1.0 / lam**2, 0.0)
    Z = transform_1d(transform_1d(X * w, bcy, axis=0, inverse=True), bcx, axis=1,
                     inverse=True)
    return np.where(known, 0.0, Z)


def pcg(known, F, bcx, bcy, tol, maxit, precond=True, flexible=False,
        precond_dtype=np.float64, x0=None):
    """Matrix-free (preconditioned) conjugate gradients on A_UU u = b, as in
    Algorithm 1: x0 = 0, stop when the recursive residual satisfies
    ||r|| <= tol ||b||.  Vectors live on the full grid and are zero at known
    nodes.  ``flexible`` uses the Polak-Ribiere form of beta,
    r_new.(z_new - z_old) / (r_old.z_old), which tolerates an inexact
    preconditioner; ``precond_dtype`` float32 runs the transforms in single
    precision.

    ``x0`` (a full grid; its values at known nodes are ignored) is a first
    iterate other than zero, the textbook generalisation of CG's start:
    r0 = b - A_UU x0, which is -(A f) at U with f = F at known nodes and x0
    at unknown ones; the stopping rule is unchanged, so a start that already
    meets it returns after 0 iterations.  A non-finite r0 raises ValueError.

    Returns (x_full, iterations, relres_history)."""
    F = np.asarray(F, dtype=np.float64)
    unknown = ~known
    f0 = np.where(known, F, 0.0)
    b = np.where(unknown, -stencil_padded(f0, bcx, bcy), 0.0)
    bnorm = np.sqrt(np.sum(b * b))
    x = np.zeros_like(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist
    r = b.copy()
    if x0 is not None:
        x = np.where(unknown, np.asarray(x0, dtype=np.float64), 0.0)
        r = np.where(unknown, -stencil_padded(np.where(known, F, x), bcx, bcy), 0.0)
        if not np.all(np.isfinite(r)):
            raise ValueError("non-finite residual of the first iterate")
        hist = [np.sqrt(np.sum(r * r)) / bnorm]
        if hist[0] <= tol:
            return x, 0, hist

    def M(v):
        if not precond:
            return v.copy()
        z = spectral_preconditioner(v.astype(precond_dtype), known, bcx, bcy)
        return np.where(unknown, z.astype(np.float64), 0.0)

    z = M(r)
    rz = np.sum(r * z)
    p = z.copy()
    for it in range(1, maxit + 1):
        q = np.where(unknown, stencil_padded(p, bcx, bcy), 0.0)
        alpha = rz / np.sum(p * q)
        x += alpha * p
        r -= alpha * q
        rel = np.sqrt(np.sum(r * r)) / bnorm
        hist.append(rel)
        if rel <= tol:
            return x, it, hist
        z_new = M(r)
        rz_new = np.sum(r * z_new)
        beta = (rz_new - np.sum(r * z)) / rz if flexible else rz_new / rz
        z, rz = z_new, rz_new
        p = z + beta * p
    return x, maxit, hist


# ----------------------------------------------------------------------------
# Metrics
# ----------------------------------------------------------------------------

def true_relative_residual(known, F_in, F_out, bcx, bcy):
    """||b - A_UU u|| / ||b|| in long double, with u = F_out at unknown nodes
    and b formed from F_in at known nodes (0 when b = 0 and u = 0)."""
    unknown = ~known
    f0 = np.asarray(np.where(known, F_in, 0.0), dtype=np.longdouble)
    b = -stencil_padded(f0, bcx, bcy)[unknown]
    f = f0.copy()
    f[unknown] = np.asarray(F_out, dtype=np.longdouble)[unknown]
    r = -stencil_padded(f, bcx, bcy)[unknown]
    bn = np.sqrt(np.sum(b * b))
    rn = np.sqrt(np.sum(r * r))
    if bn == 0:
        return float(rn)
    return float(rn / bn)


def relative_l2(a, ref):
    """||a - ref||_2 / ||ref||_2 over all nodes."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm((a - ref).ravel())
    n = np.linalg.norm(ref.ravel())
    return float(d / n) if n > 0 else float(d)
