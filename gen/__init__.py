"""Seeded synthetic inputs for the pipelined flexible Krylov solvers.

This module is shared by the FP64 oracle (``oracle/``) and by the GPU path
(``paper_1511_07226_amd``).  It produces plain numpy arrays and holds none of
the solvers' arithmetic: no operator, no preconditioner, no inner product.

Grid conventions (the same on both sides):

* ``dim`` is 2 or 3; ``n`` interior nodes per axis; mesh width h = 1/(n+1);
  node with padded index a (0..n+1) sits at coordinate a*h, so padded index 0
  and n+1 are the Dirichlet boundary.
* Node fields (``eta``, face velocities) live on the padded grid, numpy shape
  ``(n+2,)*dim`` indexed ``[z][y][x]`` (2D: ``[y][x]``), i.e. x fastest.
* Unknown vectors (``b``, ``x``) cover interior nodes only: N = n**dim values,
  x fastest.

The inputs stand in for the paper's viscous-sinker workloads (section 6.2,
3D sinker; section 6.3, 2D Stokes sinker): non-grid-aligned inclusions of
high viscosity with contrast 1e2-1e4 in a unit box.  Those application
problems (pTatin3D, PETSc ex43) are not available, so these generators stand
in for them.

Random streams: ``numpy.random.default_rng`` seeded through
``SeedSequence(seed).spawn(3)`` gives three independent streams, used for
geometry, right-hand side and velocity in that fixed role.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "streams",
    "sinker_eta",
    "rhs",
    "divfree_face_velocity",
    "make_problem",
    "config_problem",
    "batched_problems",
    "toy_diagonal",
    "study_problem",
    "graded_problem",
    "CONFIGS",
]


def streams(seed: int):
    """Three independent generators: (geometry, rhs, velocity)."""
    ss = np.random.SeedSequence(seed)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


def sinker_eta(dim: int, n: int, n_incl: int, eta_in: float, rng,
               radius=(0.05, 0.15), eta_out: float = 1.0) -> np.ndarray:
    """Piecewise-constant viscosity on the padded node grid.

    ``n_incl`` spheres (3D) or circles (2D): for each one the centre is drawn
    U[0,1]^dim (coordinates x, y[, z] in that order), then the radius
    U(radius).  A node belongs to an inclusion if its distance to the centre
    is at most the radius; overlapping inclusions are not additive.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    h = 1.0 / (n + 1)
    coords = np.arange(n + 2, dtype=np.float64) * h
    eta = np.full((n + 2,) * dim, eta_out, dtype=np.float64)
    if dim == 2:
        Y, X = np.meshgrid(coords, coords, indexing="ij")
        pts = (X, Y)
    else:
        Z, Y, X = np.meshgrid(coords, coords, coords, indexing="ij")
        pts = (X, Y, Z)
    for _ in range(n_incl):
        c = rng.uniform(0.0, 1.0, size=dim)
        r = rng.uniform(radius[0], radius[1])
        d2 = sum((p - ci) ** 2 for p, ci in zip(pts, c))
        eta[d2 <= r * r] = eta_in
    return eta


def rhs(dim: int, n: int, rng) -> np.ndarray:
    """f ~ N(0,1) on the interior nodes, flat, x fastest."""
    return rng.standard_normal(n ** dim)


def _edge_potential(dim_pts, rng, kmax: int = 2):
    """Random smooth vector potential Psi = sum_k a_k sin(2 pi k.x + phi_k).

    Wavevectors k are the nonzero integer vectors with |k|_2 <= kmax, taken in
    lexicographic order; per potential component c and wavevector k the draws
    are a ~ N(0,1)/|k|^2 and phi ~ U(0, 2 pi), component-major.
    Returns a function psi(c, X, Y, Z).
    """
    ks = []
    rng_k = range(-kmax, kmax + 1)
    for kx in rng_k:
        for ky in rng_k:
            for kz in rng_k:
                k2 = kx * kx + ky * ky + kz * kz
                if 0 < k2 <= kmax * kmax:
                    ks.append((kx, ky, kz, k2))
    coef = []
    for c in range(3):
        row = []
        for (kx, ky, kz, k2) in ks:
            a = rng.standard_normal() / k2
            phi = rng.uniform(0.0, 2.0 * math.pi)
            row.append((kx, ky, kz, a, phi))
        coef.append(row)

    def psi(c, X, Y, Z):
        out = np.zeros(np.broadcast(X, Y, Z).shape)
        for (kx, ky, kz, a, phi) in coef[c]:
            out += a * np.sin(2.0 * math.pi * (kx * X + ky * Y + kz * Z) + phi)
        return out

    def psi_grid(c, xs, ys, zs):
        """psi(c) on the tensor grid xs (x) ys (x) zs, returned as [z][y][x]:
        sin(t + phi) = Im(e^{i phi} e^{i 2 pi kx x} e^{i 2 pi ky y} e^{i 2 pi kz z}),
        summed one axis at a time (the same value as psi up to rounding)."""
        K = 2 * kmax + 1
        C3 = np.zeros((K, K, K), dtype=np.complex128)          # [kx][ky][kz]
        for (kx, ky, kz, a, phi) in coef[c]:
            C3[kx + kmax, ky + kmax, kz + kmax] += a * np.exp(1j * phi)
        kk = np.arange(-kmax, kmax + 1, dtype=np.float64)[:, None]
        Ex = np.exp(2j * math.pi * kk * np.asarray(xs)[None, :])  # [kx][x]
        Ey = np.exp(2j * math.pi * kk * np.asarray(ys)[None, :])
        Ez = np.exp(2j * math.pi * kk * np.asarray(zs)[None, :])
        T1 = np.einsum("abc,cz->abz", C3, Ez)                  # [kx][ky][z]
        T2 = np.einsum("abz,by->azy", T1, Ey)                  # [kx][z][y]
        out = np.zeros((len(zs), len(ys), len(xs)))
        for a in range(K):
            out += (T2[a][:, :, None] * Ex[a][None, None, :]).imag
        return out

    psi.grid = psi_grid

    return psi


def divfree_face_velocity(n: int, rng, cell_peclet: float = 5.0,
                          eta_bg: float = 1.0) -> np.ndarray:
    """Discretely divergence-free face-normal velocities for 3D conv-diff.

    Returns ``vel`` of shape (3, n+2, n+2, n+2): ``vel[c][k][j][i]`` is the
    velocity component along axis c (0=x, 1=y, 2=z) on the face between padded
    node (i,j,k) and its +c neighbour.  The field is the discrete curl of a
    vector potential sampled on the dual-grid edges, so the net flux out of
    every node's control volume vanishes up to rounding.  It is scaled so that
    max|v| * h / (2 * eta_bg) equals ``cell_peclet``.
    """
    h = 1.0 / (n + 1)
    psi = _edge_potential(3, rng)
    a = np.arange(n + 2, dtype=np.float64)

    def P(c, di, dj, dk):
        # potential component c at the dual edge offset by (di,dj,dk)*h/2, as [k][j][i]
        return psi.grid(c, (a + di) * h, (a + dj) * h, (a + dk) * h)

    # Psi_x on x-edges at (i, j+1/2, k+1/2); Psi_y at (i+1/2, j, k+1/2);
    # Psi_z at (i+1/2, j+1/2, k).
    vx = (P(2, 0.5, 0.5, 0.0) - P(2, 0.5, -0.5, 0.0)) - (P(1, 0.5, 0.0, 0.5) - P(1, 0.5, 0.0, -0.5))
    vy = (P(0, 0.0, 0.5, 0.5) - P(0, 0.0, 0.5, -0.5)) - (P(2, 0.5, 0.5, 0.0) - P(2, -0.5, 0.5, 0.0))
    vz = (P(1, 0.5, 0.0, 0.5) - P(1, -0.5, 0.0, 0.5)) - (P(0, 0.0, 0.5, 0.5) - P(0, 0.0, -0.5, 0.5))
    vel = np.stack([vx, vy, vz]) / h
    vmax = float(np.max(np.abs(vel)))
    if vmax > 0.0:
        vel *= (cell_peclet * 2.0 * eta_bg / h) / vmax
    return vel


@dataclass
class Problem:
    """One synthetic linear system: operator coefficients plus right-hand side."""
    dim: int
    n: int
    eta: np.ndarray                 # padded node viscosity, (n+2,)*dim
    b: np.ndarray                   # interior rhs, N
    vel: np.ndarray | None = None   # (3, n+2, n+2, n+2) face velocities or None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.dim


def make_problem(dim: int, n: int, n_incl: int, log10_contrast, seed: int,
                 convection: bool = False, cell_peclet: float = 5.0) -> Problem:
    """Sinker problem: background eta=1, inclusions at 10**contrast.

    ``log10_contrast`` is a number, or a (lo, hi) pair from which the contrast
    exponent is drawn U(lo, hi) on the geometry stream before the inclusions.
    """
    g_geo, g_rhs, g_vel = streams(seed)
    if isinstance(log10_contrast, (tuple, list)):
        c = float(g_geo.uniform(log10_contrast[0], log10_contrast[1]))
    else:
        c = float(log10_contrast)
    eta = sinker_eta(dim, n, n_incl, 10.0 ** c, g_geo)
    b = rhs(dim, n, g_rhs)
    vel = None
    if convection:
        if dim != 3:
            raise ValueError("convection inputs are 3D")
        vel = divfree_face_velocity(n, g_vel, cell_peclet=cell_peclet)
    return Problem(dim, n, eta, b, vel,
                   dict(n_incl=n_incl, log10_contrast=c, seed=seed, convection=convection))


# The five workloads.  "cfgM" is the 256^3 SPD sinker the headline throughput
# is measured on (config 2's recipe at n=256).
CONFIGS = {
    "cfg1": dict(dim=2, n=64, n_incl=8, log10_contrast=3.0, nu=30, inner_its=2, rtol=1e-8, maxit=500),
    "cfg2": dict(dim=3, n=128, n_incl=20, log10_contrast=4.0, nu=30, inner_its=5, rtol=1e-8, maxit=2000),
    "cfgM": dict(dim=3, n=256, n_incl=20, log10_contrast=4.0, nu=30, inner_its=5, rtol=1e-8, maxit=2000),
    "cfg3": dict(dim=3, n=256, n_incl=20, log10_contrast=4.0, nu=30, inner_its=5, rtol=1e-8, maxit=2000,
                 convection=True),
}


def config_problem(name: str, seed: int = 0, n: int | None = None) -> Problem:
    """Problem of a named workload; ``n`` overrides the grid size (same recipe)."""
    c = CONFIGS[name]
    return make_problem(c["dim"], n if n is not None else c["n"], c["n_incl"],
                        c["log10_contrast"], seed, convection=c.get("convection", False))


def batched_problems(count: int = 64, seed: int = 0, sizes=(32, 48, 64, 80, 96),
                     n_incl: int = 20, contrast=(2.0, 4.0)):
    """Uneven batch: edge length uniform over ``sizes``, own sinker field each.

    The size list is drawn from the first spawned stream of ``seed``; system s
    then uses seed ``seed*1000 + 1 + s`` for its own fields.
    """
    g = streams(seed)[0]
    ns = [int(sizes[i]) for i in g.integers(0, len(sizes), size=count)]
    return [make_problem(3, ns[s], n_incl, contrast, seed * 1000 + 1 + s) for s in range(count)]


def toy_diagonal(n: int = 100, cond: float = 5.0):
    """Diagonal toy system of the FCG stagnation study (section 2.2.1, Fig. 1).

    Eigenvalues equally spaced in [1, cond] (lambda_j = 1 + (cond-1) j/(n-1)),
    b = ones/sqrt(n).  Returns (diag, b).
    """
    lam = 1.0 + (cond - 1.0) * np.arange(n, dtype=np.float64) / (n - 1)
    b = np.ones(n) / math.sqrt(n)
    return lam, b


def study_problem(dim: int, n: int, seed: int = 0) -> Problem:
    """Stencil system for the noisy-preconditioner stagnation study at scale.

    The Figure 1 toy (section 2.2.1) pairs B(r) = r + noise with a spectrum of
    order one.  Constant viscosity eta = h^2 cancels the stencil's 1/h^2, so
    the operator is the unscaled Dirichlet graph Laplacian (spectrum inside
    (0, 4*dim]) and the noise of B(w - r) stays comparable to that of B(r).
    Returns the system with ``b`` a standard-normal right-hand side and the
    seeded exact solution ``x_star`` (standard normal) in ``meta``; a caller
    that needs A x_star = b forms b with its own operator.
    """
    g_geo, g_rhs, _ = streams(seed)
    h = 1.0 / (n + 1)
    eta = np.full((n + 2,) * dim, h * h, dtype=np.float64)
    b = rhs(dim, n, g_rhs)
    x_star = g_geo.standard_normal(n ** dim)
    return Problem(dim, n, eta, b, None, dict(seed=seed, x_star=x_star, study=True))


def graded_problem(dim: int, n: int, log10_range=(0.0, 4.0), seed: int = 0,
                   convection: bool = False) -> Problem:
    """System whose viscosity varies from node to node: log10(eta) drawn
    U(lo, hi) independently at every padded node, f ~ N(0, 1).

    The sinker fields take two values, so their reduced-precision copies are
    checked at two numbers only; here almost every node's value sits between
    two BF16 numbers, which makes a coefficient-rounding rule visible (the
    sinker and this field exercise the same operator).
    """
    g_geo, g_rhs, g_vel = streams(seed)
    lo, hi = log10_range
    eta = 10.0 ** g_geo.uniform(lo, hi, size=(n + 2,) * dim)
    b = rhs(dim, n, g_rhs)
    vel = divfree_face_velocity(n, g_vel) if convection else None
    return Problem(dim, n, eta, b, vel, dict(seed=seed, graded=tuple(log10_range), convection=convection))
