"""Seeded synthetic inputs: level-set functions and fields to extend.

This module only evaluates closed-form test fields on grids (it holds none of
the extension method's arithmetic), so both the GPU library's tests and the
CPU oracle can take their inputs from it.  Every generator is deterministic
given its seed.

Grid placement: Neumann and Dirichlet axes use cell-centred nodes
x_i = a + (i + 1/2) L / n (the half-sample reflection puts the boundary half a
cell outside the first node); periodic axes use x_i = a + i L / n.  Arrays are
(ny, nx), row-major with x fastest.  Only the sign of phi matters to the
method; phi is negative where the field is known.

The workload families follow the paper's examples (Sec. 3): single
interfaces (circle, star-shaped curve, two-disc peanut, annulus), multiply
connected periodic interfaces, and smooth fields (polynomials, products of
trigonometric functions, sums of Fourier modes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NEUMANN, PERIODIC, DIRICHLET = 0, 1, 2


def bc_code(bcx: int, bcy: int) -> int:
    """Per-axis boundary rule packed the way the C interface takes it."""
    return int(bcx) | (int(bcy) << 4)


@dataclass
class Problem:
    phi: np.ndarray          # (ny, nx) float64, known where phi < 0
    F: np.ndarray            # (ny, nx) float64, values used at known nodes
    bcx: int
    bcy: int
    h: float
    tol: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return int(self.phi.shape[1])

    @property
    def ny(self) -> int:
        return int(self.phi.shape[0])

    @property
    def bc(self) -> int:
        return bc_code(self.bcx, self.bcy)


def axis_nodes(n: int, a: float, b: float, bc: int) -> np.ndarray:
    """Node coordinates along one axis of [a, b] for boundary rule ``bc``."""
    L = b - a
    i = np.arange(n, dtype=np.float64)
    if bc == PERIODIC:
        return a + i * (L / n)
    return a + (i + 0.5) * (L / n)


def _mesh(nx, ny, box, bcx, bcy):
    (x0, x1), (y0, y1) = box
    x = axis_nodes(nx, x0, x1, bcx)
    y = axis_nodes(ny, y0, y1, bcy)
    return np.meshgrid(x, y)          # X[j, i] = x_i, Y[j, i] = y_j


# ----------------------------------------------------------------------------
# Fixed-shape workloads (single instances)
# ----------------------------------------------------------------------------

def circle_problem(n: int = 64, tol: float = 1e-10) -> Problem:
    """n x n on [-1, 1]^2, Neumann both axes; phi = distance to the circle of
    radius 0.5 about the origin; F = x^2 + sin(2y) known inside, extended
    outward."""
    X, Y = _mesh(n, n, ((-1, 1), (-1, 1)), NEUMANN, NEUMANN)
    phi = np.sqrt(X**2 + Y**2) - 0.5
    F = X**2 + np.sin(2 * Y)
    return Problem(phi, F, NEUMANN, NEUMANN, 2.0 / n, tol, f"circle{n}")


def star_inward_problem(n: int = 1024, tol: float = 1e-8) -> Problem:
    """n x n on [-1, 1]^2, Neumann; interface r(theta) = 0.4 (1 + 0.1 cos 5theta);
    F = exp(x) cos(3y) known OUTSIDE the star and extended inward (phi is the
    negated star function, so phi < 0 outside)."""
    X, Y = _mesh(n, n, ((-1, 1), (-1, 1)), NEUMANN, NEUMANN)
    rho = np.sqrt(X**2 + Y**2)
    th = np.arctan2(Y, X)
    star = rho - 0.4 * (1 + 0.1 * np.cos(5 * th))
    phi = -star
    F = np.exp(X) * np.cos(3 * Y)
    return Problem(phi, F, NEUMANN, NEUMANN, 2.0 / n, tol, f"star_in{n}")


def _fourier_field(X, Y, rng, modes=8, kmax=6, period=1.0):
    F = np.zeros_like(X)
    for _ in range(modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=2)
            if k[0] != 0 or k[1] != 0:
                break
        a = rng.normal()
        psi = rng.uniform(0, 2 * np.pi)
        F += a * np.cos(2 * np.pi * (k[0] * X + k[1] * Y) / period + psi)
    return F


def _circles_phi(X, Y, rng, count, rmin=0.05, rmax=0.15, periodic=True):
    """min over ``count`` circles of (distance - radius); centres uniform on
    the unit square the grids cover, radii U[rmin, rmax].  ``periodic``: the
    distance is the minimum-image one on the unit torus; otherwise plain."""
    phi = np.full(X.shape, np.inf)
    for _ in range(count):
        cx, cy = rng.uniform(0, 1, size=2)
        r = rng.uniform(rmin, rmax)
        dx = X - cx
        dy = Y - cy
        if periodic:
            dx -= np.round(dx)                     # minimum image, period 1
            dy -= np.round(dy)
        phi = np.minimum(phi, np.sqrt(dx * dx + dy * dy) - r)
    return phi


def periodic_circles_problem(n: int = 2048, seed: int = 3, circles: int = 20,
                             tol: float = 1e-8) -> Problem:
    """n x n periodic grid on [0, 1)^2; phi = min over seeded circles (centres
    uniform, radii U[0.05, 0.15], minimum-image distance) minus radius; F = 8
    seeded Fourier modes (integer wave vectors with |k|_inf <= 6, amplitudes
    N(0, 1), phases U[0, 2pi)) known inside the circles."""
    rng = np.random.default_rng(seed)
    X, Y = _mesh(n, n, ((0, 1), (0, 1)), PERIODIC, PERIODIC)
    phi = _circles_phi(X, Y, rng, circles)
    F = _fourier_field(X, Y, rng)
    return Problem(phi, F, PERIODIC, PERIODIC, 1.0 / n, tol, f"pcircles{n}",
                   {"seed": seed})


# ----------------------------------------------------------------------------
# Batched instances: star interfaces, cubic fields, mixed boundaries
# ----------------------------------------------------------------------------

def _star_phi(X, Y, rng, r0=0.5, terms=8, amax=0.05):
    a = rng.uniform(0, amax, size=terms)
    psi = rng.uniform(0, 2 * np.pi, size=terms)
    th = np.arctan2(Y, X)
    r = np.ones_like(th)
    for k in range(terms):
        r += a[k] * np.cos((k + 1) * th + psi[k])
    return np.sqrt(X**2 + Y**2) - r0 * r


def _cubic_field(X, Y, rng):
    c = rng.normal(size=10)
    return (c[0] + c[1] * X + c[2] * Y + c[3] * X * X + c[4] * X * Y + c[5] * Y * Y
            + c[6] * X**3 + c[7] * X * X * Y + c[8] * X * Y * Y + c[9] * Y**3)


def star_cubic_instance(rng, nmin=64, nmax=512, tol=1e-8) -> Problem:
    """One batched instance: nx, ny independently log-uniform in [nmin, nmax];
    spacing h = 2 / min(nx, ny) on a box centred at the origin; star-shaped
    interface r0 (1 + sum_k a_k cos(k theta + psi_k)), k <= 8, a_k ~ U[0, 0.05];
    known side inside or outside with probability 1/2; F a cubic polynomial
    with N(0, 1) coefficients; each axis Neumann or periodic with
    probability 1/2."""
    nx = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    ny = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    bcx = int(rng.integers(0, 2))
    bcy = int(rng.integers(0, 2))
    h = 2.0 / min(nx, ny)
    X, Y = _mesh(nx, ny, ((-nx * h / 2, nx * h / 2), (-ny * h / 2, ny * h / 2)), bcx, bcy)
    phi = _star_phi(X, Y, rng)
    inside = bool(rng.integers(0, 2))
    if not inside:
        phi = -phi
    F = _cubic_field(X, Y, rng)
    return Problem(phi, F, bcx, bcy, h, tol, f"star{nx}x{ny}",
                   {"known_inside": inside})


def star_cubic_batch(count: int = 256, seed: int = 4, nmin=64, nmax=512,
                     tol=1e-8) -> list:
    rng = np.random.default_rng(seed)
    return [star_cubic_instance(rng, nmin, nmax, tol) for _ in range(count)]


# ----------------------------------------------------------------------------
# Serving requests: square grids of mixed sizes and boundary types
# ----------------------------------------------------------------------------

@dataclass
class RequestSpec:
    """A request drawn from the serving mix; ``materialise`` builds its
    arrays (deterministic from ``seed``)."""
    seed: int
    n: int
    bc: int                  # NEUMANN or PERIODIC on both axes
    kind: str                # "circles" or "star"
    tol: float = 1e-8

    def params(self) -> dict:
        """The request's random parameters, drawn from its seed in a fixed
        order: the interface (circle centres and radii, or the star's
        amplitudes and phases), then the 8 Fourier modes of F."""
        rng = np.random.default_rng(self.seed)
        out = {"kind": self.kind}
        if self.kind == "circles":
            circ = []
            for _ in range(int(rng.integers(1, 21))):
                cx, cy = rng.uniform(0, 1, size=2)
                circ.append((cx, cy, rng.uniform(0.05, 0.15)))
            out["circles"] = circ
        else:
            out["star_a"] = rng.uniform(0, 0.05, size=8)
            out["star_psi"] = rng.uniform(0, 2 * np.pi, size=8)
        modes = []
        for _ in range(8):
            while True:
                k = rng.integers(-6, 7, size=2)
                if k[0] != 0 or k[1] != 0:
                    break
            modes.append((int(k[0]), int(k[1]), rng.normal(), rng.uniform(0, 2 * np.pi)))
        out["modes"] = modes
        return out

    def materialise(self) -> Problem:
        """numpy arrays on the host."""
        n, bc = self.n, self.bc
        X, Y = _mesh(n, n, ((0, 1), (0, 1)), bc, bc)
        phi, F = _request_fields(self.params(), X, Y, bc == PERIODIC, np)
        if not (phi < 0).any():          # guarantee a known node
            phi.flat[0] = -1.0
        return Problem(phi, F, bc, bc, 1.0 / n, self.tol, f"req{self.seed}")

    def materialise_torch(self, device):
        """The same fields evaluated by torch on ``device`` (float64), for
        streams too long to build on the host; the values agree with
        ``materialise`` to rounding.  Returns (phi, F) tensors."""
        import torch
        n, bc = self.n, self.bc
        x = torch.as_tensor(axis_nodes(n, 0.0, 1.0, bc), device=device)
        Y, X = torch.meshgrid(x, x, indexing="ij")          # X[j, i] = x_i
        phi, F = _request_fields(self.params(), X, Y, bc == PERIODIC, torch)
        if not bool((phi < 0).any()):
            phi.view(-1)[0] = -1.0
        return phi.contiguous(), F.contiguous()


def _request_fields(prm, X, Y, periodic, xp):
    """phi and F of a serving request from its parameters, with array module
    ``xp`` (numpy or torch): the multi-circle or star interface, known
    inside, and the sum of Fourier modes."""
    if prm["kind"] == "circles":
        phi = None
        for cx, cy, r in prm["circles"]:
            dx = X - cx
            dy = Y - cy
            if periodic:
                dx = dx - xp.round(dx)                     # minimum image, period 1
                dy = dy - xp.round(dy)
            d = xp.sqrt(dx * dx + dy * dy) - r
            phi = d if phi is None else xp.minimum(phi, d)
    else:
        Xc, Yc = X - 0.5, Y - 0.5
        th = xp.arctan2(Yc, Xc)
        rr = xp.ones_like(th)
        for k in range(8):
            rr = rr + prm["star_a"][k] * xp.cos((k + 1) * th + prm["star_psi"][k])
        phi = xp.sqrt(Xc * Xc + Yc * Yc) - 0.25 * rr
    F = xp.zeros_like(X)
    for kx, ky, a, psi in prm["modes"]:
        F = F + a * xp.cos(2 * np.pi * (kx * X + ky * Y) + psi)
    return phi, F


def request_stream(count: int = 10000, seed: int = 5, nmin=128, nmax=2048,
                   tol=1e-8) -> list:
    """Request specs: side log-uniform in [nmin, nmax]; Neumann or periodic
    (1/2 each); multi-circle (1-20 circles) or star interface (1/2 each);
    Fourier-mode field known inside."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        bc = NEUMANN if rng.integers(0, 2) == 0 else PERIODIC
        kind = "circles" if rng.integers(0, 2) == 0 else "star"
        out.append(RequestSpec(int(rng.integers(0, 2**31 - 1)), n, bc, kind, tol))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 6) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of ``rate``/s."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# ----------------------------------------------------------------------------
# The paper's own examples (Sec. 3.1 and 3.3), used for calibration
# ----------------------------------------------------------------------------

def peanut_problem(n: int, bcx: int, bcy: int, tol: float = 1e-6) -> Problem:
    """Example 1: D = [-pi, pi]^2, f = cos x sin y known inside the union of
    two unit discs centred at (+-0.8, 0)."""
    X, Y = _mesh(n, n, ((-np.pi, np.pi), (-np.pi, np.pi)), bcx, bcy)
    phi = np.minimum(np.sqrt((X - 0.8) ** 2 + Y**2) - 1, np.sqrt((X + 0.8) ** 2 + Y**2) - 1)
    F = np.cos(X) * np.sin(Y)
    return Problem(phi, F, bcx, bcy, 2 * np.pi / n, tol, f"peanut{n}")


def annulus_problem(n: int, bcx: int, bcy: int, tol: float = 1e-6) -> Problem:
    """Example 3: D = [-2, 2]^2, f = y / log(1 + r) known in 1/2 < r < 1."""
    X, Y = _mesh(n, n, ((-2, 2), (-2, 2)), bcx, bcy)
    r = np.sqrt(X**2 + Y**2)
    phi = np.maximum(0.5 - r, r - 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(r > 0, Y / np.log1p(r), 0.0)
    return Problem(phi, F, bcx, bcy, 4.0 / n, tol, f"annulus{n}")


def channel_problem(ny: int, terms: int = 10, seed: int = 8, bcy: int = PERIODIC,
                    tol: float = 1e-6) -> Problem:
    """Example 4 (Sec. 3.4): D = [0, 3] x [0, 1] on a 3 ny x ny grid, Neumann
    sides, periodic (or, for the channel geometry, Neumann) top and bottom.
    The interface is x = 1.5 + sum_k a_k sin(2 pi k y + w_k), k = 1..terms,
    with seeded a_k ~ U[-0.05, 0.05] and w_k ~ U[0, 2 pi); f is known to the
    left of it: x + cos(2 pi (y - 1/4)) / 5 with periodic top and bottom,
    x + cos(pi y) / 5 with Neumann ones."""
    nx = 3 * ny
    X, Y = _mesh(nx, ny, ((0.0, 3.0), (0.0, 1.0)), NEUMANN, bcy)
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.05, 0.05, size=terms)
    w = rng.uniform(0.0, 2 * np.pi, size=terms)
    front = 1.5 + sum(a[k] * np.sin(2 * np.pi * (k + 1) * Y + w[k]) for k in range(terms))
    phi = X - front
    if bcy == PERIODIC:
        F = X + np.cos(2 * np.pi * (Y - 0.25)) / 5
    else:
        F = X + np.cos(np.pi * Y) / 5
    return Problem(phi, F, NEUMANN, bcy, 1.0 / ny, tol, f"channel{nx}x{ny}",
                   {"amplitudes": a, "phases": w})


# ----------------------------------------------------------------------------
# Three dimensions (Sec. 3.2, Example 2)
# ----------------------------------------------------------------------------

def bc_code3(bcx: int, bcy: int, bcz: int) -> int:
    """Per-axis boundary rules of a 3-D problem packed for the C interface."""
    return int(bcx) | (int(bcy) << 4) | (int(bcz) << 8)


@dataclass
class Problem3:
    phi: np.ndarray          # (nz, ny, nx) float64, known where phi < 0
    F: np.ndarray            # (nz, ny, nx) float64, values used at known nodes
    bcx: int
    bcy: int
    bcz: int
    h: float
    tol: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return int(self.phi.shape[2])

    @property
    def ny(self) -> int:
        return int(self.phi.shape[1])

    @property
    def nz(self) -> int:
        return int(self.phi.shape[0])

    @property
    def bc(self) -> int:
        return bc_code3(self.bcx, self.bcy, self.bcz)


def _mesh3(nx, ny, nz, box, bcx, bcy, bcz):
    (x0, x1), (y0, y1), (z0, z1) = box
    z, y, x = (axis_nodes(nz, z0, z1, bcz), axis_nodes(ny, y0, y1, bcy),
               axis_nodes(nx, x0, x1, bcx))
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")     # X[k, j, i] = x_i
    return X, Y, Z


def peanut3d_problem(n: int, bcx: int = PERIODIC, bcy: int = PERIODIC, bcz: int = PERIODIC,
                     tol: float = 1e-6) -> Problem3:
    """Example 2: D = [-pi, pi]^3, f = cos x sin y sin(pi/4 - z) known inside
    the union of two unit balls centred at (+-0.8, 0, 0); periodic in the
    paper."""
    box = ((-np.pi, np.pi),) * 3
    X, Y, Z = _mesh3(n, n, n, box, bcx, bcy, bcz)
    phi = np.minimum(np.sqrt((X - 0.8) ** 2 + Y**2 + Z**2) - 1,
                     np.sqrt((X + 0.8) ** 2 + Y**2 + Z**2) - 1)
    F = np.cos(X) * np.sin(Y) * np.sin(np.pi / 4 - Z)
    return Problem3(phi, F, bcx, bcy, bcz, 2 * np.pi / n, tol, f"peanut3d_{n}")


def ball_problem3(nx: int, ny: int, nz: int, bcx: int, bcy: int, bcz: int, seed: int = 0,
                  tol: float = 1e-10, inside: bool = True) -> Problem3:
    """[-1, 1]^3 with a ball of radius U[0.3, 0.45] about a random centre
    within 0.2 of the origin; F a random cubic plus sin(2y) cos(z); known
    inside the ball (or outside it)."""
    rng = np.random.default_rng(seed)
    X, Y, Z = _mesh3(nx, ny, nz, ((-1, 1),) * 3, bcx, bcy, bcz)
    c = rng.uniform(-0.2, 0.2, size=3)
    rad = rng.uniform(0.3, 0.45)
    phi = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - rad
    if not inside:
        phi = -phi
    a = rng.normal(size=6)
    F = (a[0] * X**3 + a[1] * X * Y * Z + a[2] * Y**2 + a[3] * Z + a[4]
         + a[5] * np.sin(2 * Y) * np.cos(Z))
    return Problem3(phi, F, bcx, bcy, bcz, 2.0 / max(nx, ny, nz), tol,
                    f"ball{nx}x{ny}x{nz}")
