"""Pins for the oracle's inner-solve preconditioners (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import gen
from oracle import StencilOperator, jacobi_pcg, jacobi_gmres


def _problem(dim=2, n=10, contrast=2.0, seed=1):
    p = gen.make_problem(dim, n, 3, contrast, seed)
    return StencilOperator(dim, n, p.eta, p.vel), p


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_jacobi_pcg_matches_scipy_cg(k):
    A, _ = _problem()
    Dinv = 1.0 / A.diagonal()
    v = np.random.default_rng(k).standard_normal(A.N)
    L = spla.LinearOperator((A.N, A.N), matvec=A.apply, dtype=np.float64)
    M = spla.LinearOperator((A.N, A.N), matvec=lambda t: Dinv * t, dtype=np.float64)
    ref, _ = spla.cg(L, v, x0=np.zeros(A.N), rtol=0.0, atol=0.0, maxiter=k, M=M)
    y = jacobi_pcg(A.apply, Dinv, v, k)
    assert np.allclose(y, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_jacobi_pcg_one_step_closed_form():
    A, _ = _problem(3, 5)
    Dinv = 1.0 / A.diagonal()
    v = np.random.default_rng(0).standard_normal(A.N)
    z = Dinv * v
    expect = (np.dot(v, z) / np.dot(z, A.apply(z))) * z
    assert np.allclose(jacobi_pcg(A.apply, Dinv, v, 1), expect, rtol=1e-13)


def test_jacobi_pcg_exact_after_distinct_eigenvalues():
    # A with three distinct eigenvalues and M = I: three CG steps solve exactly
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    lam = np.repeat([1.0, 3.0, 7.0], 4)
    Amat = (Q * lam) @ Q.T
    v = rng.standard_normal(12)
    y = jacobi_pcg(lambda t: Amat @ t, np.ones(12), v, 3)
    assert np.allclose(y, np.linalg.solve(Amat, v), rtol=1e-10)


def test_jacobi_pcg_zero_input():
    A, _ = _problem()
    assert not np.any(jacobi_pcg(A.apply, 1.0 / A.diagonal(), np.zeros(A.N), 3))


@pytest.mark.parametrize("k,conv", [(1, False), (3, False), (5, True)])
def test_jacobi_gmres_is_minimum_residual(k, conv):
    dim = 3 if conv else 2
    n = 6 if conv else 9
    p = gen.make_problem(dim, n, 2, 1.0, seed=3, convection=conv)
    A = StencilOperator(dim, n, p.eta, p.vel)
    Dinv = 1.0 / A.diagonal()
    v = np.random.default_rng(k).standard_normal(A.N)
    # explicit Krylov basis of A D^-1 started at v (columns normalised only)
    K = [v / np.linalg.norm(v)]
    for _ in range(k - 1):
        t = A.apply(Dinv * K[-1])
        K.append(t / np.linalg.norm(t))
    K = np.array(K).T
    AK = np.array([A.apply(Dinv * K[:, j]) for j in range(k)]).T
    c = np.linalg.lstsq(AK, v, rcond=None)[0]
    expect = Dinv * (K @ c)
    y = jacobi_gmres(A.apply, Dinv, v, k)
    assert np.linalg.norm(y - expect) <= 1e-9 * np.linalg.norm(expect)
    # and its residual is no larger than the one-step (k=1) minimiser's
    r = np.linalg.norm(v - A.apply(y))
    r1 = np.linalg.norm(v - A.apply(jacobi_gmres(A.apply, Dinv, v, 1)))
    assert r <= r1 * (1 + 1e-12)


def test_jacobi_gmres_zero_input():
    A, _ = _problem()
    assert not np.any(jacobi_gmres(A.apply, 1.0 / A.diagonal(), np.zeros(A.N), 3))


@pytest.mark.parametrize("k", [1, 2, 5, 8])
def test_jacobi_gmres_exact_breakdown_one_node(k):
    # one node with eta = 1 in 2D (h = 1/2): A = 4 * 4 = 16 and A D^-1 = 1, so
    # the Krylov space is span{v}; every k returns the exact solution
    # t = v of A D^-1 t = v, i.e. B(v) = v / 16 (a zero second basis vector
    # must end the cycle cleanly, not divide by its zero norm)
    p = gen.make_problem(2, 1, 1, 1.0, seed=0)
    A = StencilOperator(2, 1, np.ones_like(p.eta))
    assert A.apply(np.array([1.0]))[0] == 16.0
    for v in (1.0, -3.0, 0.5):
        y = jacobi_gmres(A.apply, 1.0 / A.diagonal(), np.array([v]), k)
        assert np.isfinite(y).all() and abs(y[0] - v / 16.0) <= 1e-15 * abs(v)


@pytest.mark.parametrize("dim,n,bs,k,conv", [(2, 11, 4, 3, False), (3, 7, 3, 5, False), (3, 6, 4, 2, True)])
def test_block_jacobi_pcg_matches_per_block_scipy_cg(dim, n, bs, k, conv):
    from oracle import block_jacobi_pcg
    p = gen.make_problem(dim, n, 2, 3.0, seed=k, convection=conv)
    A = StencilOperator(dim, n, p.eta, p.vel)
    Dinv = 1.0 / A.diagonal()
    Adense = np.array([A.apply(e) for e in np.eye(A.N)]).T
    v = np.random.default_rng(5).standard_normal(A.N)
    y = block_jacobi_pcg(A, Dinv, v, k, bs)
    # principal submatrices of the assembled operator, one block at a time
    coords = np.array(np.unravel_index(np.arange(A.N), (n,) * dim)).T // bs
    keys = [tuple(c) for c in coords]
    expect = np.zeros(A.N)
    for key in sorted(set(keys)):
        idx = np.array([i for i, kk in enumerate(keys) if kk == key])
        Abb = Adense[np.ix_(idx, idx)]
        if conv:
            # nonsymmetric blocks: run the same PCG recurrence by hand on the dense block
            yb = np.zeros(len(idx)); r = v[idx].copy(); z = Dinv[idx] * r; pp = z.copy(); g = r @ z
            for j in range(1, k + 1):
                q = Abb @ pp; a = g / (pp @ q); yb += a * pp
                if j < k:
                    r -= a * q; z = Dinv[idx] * r; gn = r @ z; pp = z + gn / g * pp; g = gn
            expect[idx] = yb
        else:
            M = spla.LinearOperator(Abb.shape, matvec=lambda t, d=Dinv[idx]: d * t, dtype=np.float64)
            # CG is exact after len(idx) steps; scipy has no zero-residual guard, so stop there
            expect[idx], _ = spla.cg(Abb, v[idx], x0=np.zeros(len(idx)), rtol=0.0, atol=0.0,
                                     maxiter=min(k, len(idx)), M=M)
    assert np.allclose(y, expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())


def test_block_jacobi_single_block_is_global():
    from oracle import block_jacobi_pcg
    A, _ = _problem(3, 6)
    Dinv = 1.0 / A.diagonal()
    v = np.random.default_rng(2).standard_normal(A.N)
    assert np.allclose(block_jacobi_pcg(A, Dinv, v, 4, 6), jacobi_pcg(A.apply, Dinv, v, 4), rtol=1e-12)
