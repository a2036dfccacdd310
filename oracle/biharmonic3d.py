"""Plain CPU reference for the masked discrete biharmonic extension in three
dimensions.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run this module; the
GPU library never does.  It shares no code, table or helper with the HIP
path.

What it computes.  Example 2 of Sec. 3 extends the method to three
dimensions and states that the two-dimensional construction carries over
unchanged.  Written out:

* the negative 7-point Laplacian L = I (x) I (x) T_x + I (x) T_y (x) I +
  T_z (x) I (x) I, with the 1-D second difference T of each axis and its ghost
  rule (the same three rules as in 2-D, Algorithm 1);
* A = L^2, the 25-point discrete biharmonic operator (interior coefficients
  42 at the node, -12 at the six axis neighbours, +2 at the twelve in-plane
  diagonals, +1 two nodes away along an axis);
* known nodes where phi < 0, the unknowns solve A_UU u = -A_UK f_K (SPD);
* the preconditioner divides by (lambda_x + lambda_y + lambda_z)^2 in the
  tensor eigenbasis; for periodic axes the paper uses the discrete Fourier
  transform, taken here as the Hartley transform, as in 2-D.

Arrays are (nz, ny, nx), x fastest: node (i, j, k) is a[k, j, i], linear
index (k*ny + j)*nx + i.  Each function states the passage it follows.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .biharmonic import (DIRICHLET, SingularProblem, _pad_axis, eigenvalues_1d,
                         known_mask, second_difference_1d, transform_1d)

__all__ = ["laplacian_3d", "biharmonic_matrix_3d", "stencil_padded_3d", "rhs_3d",
           "reduced_system_3d", "extend_direct_3d", "spectral_preconditioner_3d", "pcg_3d",
           "true_relative_residual_3d", "known_mask"]


def laplacian_3d(nx, ny, nz, bcx, bcy, bcz):
    """Negative 7-point Laplacian as a Kronecker sum (Sec. 3, Example 2, with
    the 1-D ghost rules of Algorithm 1), row-major with x fastest."""
    Tx = second_difference_1d(nx, bcx)
    Ty = second_difference_1d(ny, bcy)
    Tz = second_difference_1d(nz, bcz)
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(Iz, sp.kron(Iy, Tx)) + sp.kron(Iz, sp.kron(Ty, Ix))
            + sp.kron(Tz, sp.kron(Iy, Ix))).tocsr()


def biharmonic_matrix_3d(nx, ny, nz, bcx, bcy, bcz):
    """Full-grid 25-point operator A = L^2 (sparse CSR, integer entries)."""
    L = laplacian_3d(nx, ny, nz, bcx, bcy, bcz)
    return (L @ L).tocsr()


def _seven_point(P):
    """6 c - (six axis neighbours) on the interior of padded array P."""
    c = P[1:-1, 1:-1, 1:-1]
    return (6 * c - P[:-2, 1:-1, 1:-1] - P[2:, 1:-1, 1:-1] - P[1:-1, :-2, 1:-1]
            - P[1:-1, 2:, 1:-1] - P[1:-1, 1:-1, :-2] - P[1:-1, 1:-1, 2:])


def stencil_padded_3d(f, bcx, bcy, bcz):
    """A f at every node, formed as Algorithm 1 forms it in 2-D: two ghost
    layers per side of each axis by that axis' rule, the 7-point Laplacian on
    the one-layer ring, then again on the grid.  Works in the dtype of f."""
    f = np.asarray(f)
    P = _pad_axis(_pad_axis(_pad_axis(f, 0, bcz), 1, bcy), 2, bcx)
    return _seven_point(_seven_point(P))


def rhs_3d(F, known, bcx, bcy, bcz):
    """b = -(A f_K) at the unknown nodes, f_K = F at known nodes and 0 at the
    others (the first step of Algorithm 1), as a vector in row-major order."""
    f = np.where(known, F, 0.0)
    return -stencil_padded_3d(f, bcx, bcy, bcz)[~known]


def reduced_system_3d(known, bcx, bcy, bcz):
    """A_UU: rows and columns of A at the unknown nodes (CSC)."""
    nz, ny, nx = known.shape
    A = biharmonic_matrix_3d(nx, ny, nz, bcx, bcy, bcz)
    U = np.flatnonzero(~known.ravel())
    return A[U][:, U].tocsc()


def extend_direct_3d(phi, F, bcx, bcy, bcz, refine=2, known=None):
    """Extension by sparse direct factorisation (the direct route of Sec. 2.2
    in three dimensions), then ``refine`` steps of iterative refinement with a
    long-double residual from the padded stencil.  Returns (F_out, info)."""
    F = np.asarray(F, dtype=np.float64)
    if known is None:
        known = known_mask(phi)
    unknown = ~known
    F_out = F.copy()
    info = {"n_unknown": int(unknown.sum()), "refine_residuals": []}
    if not unknown.any():
        return F_out, info
    if not known.any() and DIRICHLET not in (bcx, bcy, bcz):
        raise SingularProblem("no known node and no Dirichlet axis")
    b = rhs_3d(F, known, bcx, bcy, bcz)
    lu = spla.splu(reduced_system_3d(known, bcx, bcy, bcz), permc_spec="MMD_AT_PLUS_A",
                   diag_pivot_thresh=0.0, options={"SymmetricMode": True})
    u = np.asarray(lu.solve(b), dtype=np.longdouble)
    f_ld = np.asarray(np.where(known, F, 0.0), dtype=np.longdouble)
    b_norm = float(np.linalg.norm(b))
    for _ in range(refine):
        f_ld[unknown] = u
        r = -stencil_padded_3d(f_ld, bcx, bcy, bcz)[unknown]
        info["refine_residuals"].append(
            float(np.sqrt(np.sum(r * r))) / b_norm if b_norm > 0 else 0.0)
        u = u + np.asarray(lu.solve(np.asarray(r, dtype=np.float64)), dtype=np.longdouble)
    F_out[unknown] = np.asarray(u, dtype=np.float64)
    return F_out, info


def spectral_preconditioner_3d(r, known, bcx, bcy, bcz):
    """z = R T^T diag(1/Lambda^2) T R^T r in three dimensions: zero the known
    nodes, transform along x, y, z, divide by (lambda_x + lambda_y +
    lambda_z)^2 (zero where that vanishes), transform back, restrict."""
    nz, ny, nx = r.shape
    X = np.where(known, 0.0, r)
    X = transform_1d(transform_1d(transform_1d(X, bcx, axis=2), bcy, axis=1), bcz, axis=0)
    lam = (eigenvalues_1d(nz, bcz)[:, None, None] + eigenvalues_1d(ny, bcy)[None, :, None]
           + eigenvalues_1d(nx, bcx)[None, None, :])
    with np.errstate(divide="ignore"):
        w = np.where(lam > 0, 1.0 / lam**2, 0.0)
    Z = transform_1d(X * w, bcz, axis=0, inverse=True)
    Z = transform_1d(transform_1d(Z, bcy, axis=1, inverse=True), bcx, axis=2, inverse=True)
    return np.where(known, 0.0, Z)


def pcg_3d(known, F, bcx, bcy, bcz, tol, maxit, precond=True, x0=None):
    """Preconditioned conjugate gradients on A_UU u = b in three dimensions,
    as Algorithm 1 (x0 = 0 unless given; stop when the recursive residual
    satisfies ||r|| <= tol ||b||).  Vectors are full grids, zero at known
    nodes.  Returns (x_full, iterations, relres_history)."""
    F = np.asarray(F, dtype=np.float64)
    unknown = ~known

    def A(v):
        return np.where(unknown, stencil_padded_3d(v, bcx, bcy, bcz), 0.0)

    def M(v):
        if not precond:
            return v.copy()
        return spectral_preconditioner_3d(v, known, bcx, bcy, bcz)

    b = np.where(unknown, -stencil_padded_3d(np.where(known, F, 0.0), bcx, bcy, bcz), 0.0)
    bnorm = np.sqrt(np.sum(b * b))
    x = np.zeros_like(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, 0, hist
    r = b.copy()
    if x0 is not None:
        x = np.where(unknown, np.asarray(x0, dtype=np.float64), 0.0)
        r = b - A(x)
        hist = [np.sqrt(np.sum(r * r)) / bnorm]
        if hist[0] <= tol:
            return x, 0, hist
    z = M(r)
    rz = np.sum(r * z)
    p = z.copy()
    for it in range(1, maxit + 1):
        q = A(p)
        alpha = rz / np.sum(p * q)
        x += alpha * p
        r -= alpha * q
        rel = np.sqrt(np.sum(r * r)) / bnorm
        hist.append(rel)
        if rel <= tol:
            return x, it, hist
        z = M(r)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist


def true_relative_residual_3d(known, F_in, F_out, bcx, bcy, bcz):
    """||b - A_UU u|| / ||b|| in long double, u = F_out at unknown nodes and
    b from F_in at known nodes."""
    unknown = ~known
    f0 = np.asarray(np.where(known, F_in, 0.0), dtype=np.longdouble)
    b = -stencil_padded_3d(f0, bcx, bcy, bcz)[unknown]
    f = f0.copy()
    f[unknown] = np.asarray(F_out, dtype=np.longdouble)[unknown]
    r = -stencil_padded_3d(f, bcx, bcy, bcz)[unknown]
    bn = np.sqrt(np.sum(b * b))
    rn = np.sqrt(np.sum(r * r))
    return float(rn / bn) if bn > 0 else float(rn)
