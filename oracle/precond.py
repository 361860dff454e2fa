"""Flexible (nonlinear) preconditioners B, FP64, plain numpy.

Test infrastructure (see the package docstring).

The paper's experiments precondition with a few iterations of an inner Krylov
solve (section 6.2: five iterations of Jacobi-preconditioned CG per block;
section 1.1: a nested Krylov solve is a nonlinear operation).  Here the
inner solves act on the global operator:

* ``jacobi_pcg(A, v, k)``: k iterations of PCG (Alg. 3) with M = diag(A),
  from a zero initial guess, returning the iterate.  Guards: a zero
  preconditioned residual returns 0; a non-positive curvature <p, Ap>
  returns the current iterate.
  Pins: scipy.sparse.linalg.cg with the same M, x0 = 0 and maxiter = k; the
  k = 1 closed form; exact inverse once k reaches the number of distinct
  eigenvalues of D^-1 A.
* ``jacobi_gmres(A, v, k)``: one GMRES(k) cycle on A D^-1 t = v from t = 0,
  classical Gram-Schmidt Arnoldi, least squares on the Hessenberg matrix,
  returning y = D^-1 t.
  Pin: the minimiser of ||v - A D^-1 t|| over the Krylov space, computed with
  lstsq on an explicit (non-orthogonalised) basis.
* ``block_jacobi_pcg(A, v, k, bs)``: the block-Jacobi form of the paper's
  experiments: k Jacobi-PCG iterations inside every cubic block of bs nodes,
  on the block's principal submatrix, all blocks independent.
  Pins: a loop over blocks running scipy's CG on each dense block matrix;
  one block covering the grid reduces to ``jacobi_pcg``.
* ``noisy_pc``: the section 2.2.1 (Fig. 1) toy preconditioner
  B(r) = r + eta ||r|| g/||g||, g ~ N(0, I) drawn from a generator the caller
  passes in.  Parity unpinned beyond its definition (it has no GPU twin).
"""
from __future__ import annotations

import numpy as np


def _dot(a, b) -> float:
    return float(np.dot(a, b))


def identity_pc(v):
    """B = I."""
    return np.array(v, dtype=np.float64, copy=True)


def jacobi_pc(Dinv):
    """Linear Jacobi preconditioner v -> D^-1 v."""
    def B(v):
        return Dinv * v
    return B


def jacobi_pcg(A, Dinv, v, k: int):
    """k iterations of Jacobi-preconditioned CG (Alg. 3) on A y = v from y = 0."""
    y = np.zeros_like(v)
    r = np.array(v, dtype=np.float64, copy=True)
    z = Dinv * r
    p = z.copy()
    gamma = _dot(r, z)
    if gamma == 0.0:
        return y
    for j in range(1, k + 1):
        q = A(p)
        pq = _dot(p, q)
        if not pq > 0.0:
            return y
        alpha = gamma / pq
        y = y + alpha * p
        if j < k:
            r = r - alpha * q
            z = Dinv * r
            gamma_new = _dot(r, z)
            p = z + (gamma_new / gamma) * p
            gamma = gamma_new
    return y


def jacobi_gmres(A, Dinv, v, k: int):
    """One GMRES(k) cycle, right-preconditioned by D^-1, from zero; returns D^-1 t."""
    beta = float(np.linalg.norm(v))
    if beta == 0.0:
        return np.zeros_like(v)
    V = [np.asarray(v, dtype=np.float64) / beta]
    H = np.zeros((k + 1, k))
    cols = k
    for j in range(k):
        w = A(Dinv * V[j])
        for i in range(j + 1):                 # classical Gram-Schmidt: all against the same w
            H[i, j] = _dot(V[i], w)
        for i in range(j + 1):
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] == 0.0:                 # happy breakdown: the space is invariant
            cols = j + 1
            break
        if j + 1 < k:
            V.append(w / H[j + 1, j])
    rhs = np.zeros(cols + 1)
    rhs[0] = beta
    c = np.linalg.lstsq(H[:cols + 1, :cols], rhs, rcond=None)[0]
    t = np.zeros_like(V[0])
    for j in range(cols):
        t = t + c[j] * V[j]
    return Dinv * t


def _block_ids(n: int, dim: int, bs: int) -> np.ndarray:
    """Block index of every interior node (flat, x fastest) for cubic blocks of bs nodes."""
    nb = (n + bs - 1) // bs
    blk = np.arange(n) // bs
    ids = np.zeros((n,) * dim, dtype=np.int64)
    for g in np.meshgrid(*([blk] * dim), indexing="ij"):
        ids = ids * nb + g
    return ids.reshape(-1)


def block_operator(A, bs: int):
    """v -> A_bb v for every block at once: A with couplings between blocks dropped.

    Blocks are cubes of ``bs`` nodes per axis starting at interior index 0
    (the last block per axis is ragged when bs does not divide n); the
    diagonal keeps every face, so D is that of A.
    """
    n, dim, h = A.n, A.dim, A.h
    pos = np.arange(n)
    blk = pos // bs
    c0 = (slice(1, n + 1),) * dim

    def same_block(axis, sgn):
        j = pos + sgn
        ok = (j >= 0) & (j < n) & (blk == np.clip(j, 0, n - 1) // bs)
        shape = [1] * dim
        shape[axis] = n
        return ok.reshape(shape)

    def apply(u):
        U = np.zeros((n + 2,) * dim)
        U[c0] = u.reshape((n,) * dim)
        uc = U[c0]
        ec = A.eta[c0]
        y = np.zeros((n,) * dim)
        for axis, c, sgn in A._faces():
            nb = A._sl(axis, sgn)
            mask = same_block(axis, sgn)
            k = 2.0 * ec * A.eta[nb] / (ec + A.eta[nb])
            y += k * (uc - mask * U[nb]) / (h * h)
            if A.vel is not None:
                vn = A._outward_velocity(c, sgn, axis)
                y += (np.maximum(vn, 0.0) * uc + np.minimum(vn, 0.0) * mask * U[nb]) / h
        return y.reshape(-1)

    return apply


def block_jacobi_pcg(A, Dinv, v, k: int, bs: int):
    """Block-Jacobi preconditioner with k Jacobi-PCG iterations inside every block.

    The paper's experiments (section 6.2) apply, per block of the domain,
    five iterations of Jacobi-preconditioned CG from zero.  Here every cubic
    block of ``bs`` nodes per axis runs ``jacobi_pcg`` on its own principal
    submatrix A_bb with its own scalars; all blocks advance together.
    Guards per block as in ``jacobi_pcg``.
    Pin: an explicit loop over blocks running scipy's CG on the dense A_bb.
    """
    ids = _block_ids(A.n, A.dim, bs)
    nblk = int(ids.max()) + 1
    Abb = block_operator(A, bs)

    def bdot(a, b):
        return np.bincount(ids, weights=a * b, minlength=nblk)

    y = np.zeros_like(v)
    r = np.array(v, dtype=np.float64, copy=True)
    z = Dinv * r
    p = z.copy()
    gamma = bdot(r, z)
    live = gamma != 0.0
    for j in range(1, k + 1):
        q = Abb(p)
        pq = bdot(p, q)
        live = live & (pq > 0.0)
        alpha = np.where(live, gamma / np.where(live, pq, 1.0), 0.0)
        y = y + alpha[ids] * p
        if j < k:
            r = r - alpha[ids] * q
            z = Dinv * r
            gamma_new = bdot(r, z)
            beta = np.where(live, gamma_new / np.where(live, gamma, 1.0), 0.0)
            p = z + beta[ids] * p
            gamma = gamma_new
    return y


def noisy_pc(eta: float, rng):
    """Toy preconditioner of the stagnation study: r + eta*||r||*g/||g||."""
    def B(r):
        g = rng.standard_normal(r.shape[0])
        return r + eta * float(np.linalg.norm(r)) * g / float(np.linalg.norm(g))
    return B


def make_pc(kind: str, A, k: int = 0, block: int = 8):
    """Preconditioner callable by name.

    'none', 'jacobi', 'jacobi_pcg', 'jacobi_gmres', 'block_jacobi_pcg'
    (``block`` nodes per axis).
    """
    if kind == "none":
        return identity_pc
    Dinv = 1.0 / A.diagonal()
    if kind == "jacobi":
        return jacobi_pc(Dinv)
    if kind == "jacobi_pcg":
        return lambda v: jacobi_pcg(A, Dinv, v, k)
    if kind == "jacobi_gmres":
        return lambda v: jacobi_gmres(A, Dinv, v, k)
    if kind == "block_jacobi_pcg":
        return lambda v: block_jacobi_pcg(A, Dinv, v, k, block)
    raise ValueError(kind)
