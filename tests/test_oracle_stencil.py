"""Pins for the oracle's stencil operators (CPU only).

Each check pins the oracle against something other than itself: a textbook
matrix assembled independently with scipy.sparse, closed-form eigenpairs, a
hand-evaluated row, structural identities (symmetry, zero flux divergence,
transposition under velocity reversal) and a node-by-node loop.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from oracle import StencilOperator, harmonic_face


def _laplacian(dim, n):
    h = 1.0 / (n + 1)
    L1 = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / (h * h)
    I = sp.identity(n)
    if dim == 2:
        return (sp.kron(I, L1) + sp.kron(L1, I)).tocsr()
    return (sp.kron(sp.kron(I, I), L1) + sp.kron(sp.kron(I, L1), I) + sp.kron(sp.kron(L1, I), I)).tocsr()


@pytest.mark.parametrize("dim,n", [(2, 7), (2, 12), (3, 5), (3, 9)])
def test_constant_eta_is_textbook_laplacian(dim, n):
    A = StencilOperator(dim, n, np.ones((n + 2,) * dim))
    L = _laplacian(dim, n)
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = rng.standard_normal(n ** dim)
        ref = L @ u
        assert np.allclose(A.apply(u), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n", [(2, 10), (3, 6)])
def test_sine_modes_are_eigenvectors(dim, n):
    h = 1.0 / (n + 1)
    A = StencilOperator(dim, n, np.ones((n + 2,) * dim))
    idx = np.arange(1, n + 1)
    for modes in [(1,) * dim, (2, 3, 1)[:dim], (n, 1, 2)[:dim]]:
        # arrays are [z][y][x]; modes are given in x, y, z order
        comps = [np.sin(m * math.pi * idx * h) for m in modes]
        if dim == 2:
            u = np.outer(comps[1], comps[0])
        else:
            u = np.einsum("k,j,i->kji", comps[2], comps[1], comps[0])
        lam = 4.0 / (h * h) * sum(math.sin(m * math.pi * h / 2) ** 2 for m in modes)
        Au = A.apply(u.ravel())
        assert np.allclose(Au, lam * u.ravel(), rtol=1e-12, atol=1e-12 * lam)


def test_hand_evaluated_row():
    # 2D, n=3, eta = 1 except the centre padded node (2,2) which has eta = 3.
    n, h = 3, 0.25
    eta = np.ones((5, 5))
    eta[2, 2] = 3.0
    A = StencilOperator(2, n, eta)
    # face coefficient between eta=1 and eta=3 is 2*3/4 = 1.5
    assert harmonic_face(1.0, 3.0) == 1.5
    e = np.zeros(9)
    e[4] = 1.0                   # interior centre node
    col = A.apply(e)
    assert col[4] == pytest.approx(4 * 1.5 / h ** 2, rel=1e-15)
    for nb in (1, 3, 5, 7):      # its four neighbours couple through k = 1.5
        assert col[nb] == pytest.approx(-1.5 / h ** 2, rel=1e-15)
    e = np.zeros(9)
    e[0] = 1.0                   # corner node: 4 faces with k = 1 (two to the boundary)
    col = A.apply(e)
    assert col[0] == pytest.approx(4.0 / h ** 2, rel=1e-15)
    assert col[1] == pytest.approx(-1.0 / h ** 2, rel=1e-15)
    assert col[3] == pytest.approx(-1.0 / h ** 2, rel=1e-15)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_diffusion_is_symmetric_with_positive_diagonal(dim, n):
    p = gen.make_problem(dim, n, 4, 3.0, seed=5)
    A = StencilOperator(dim, n, p.eta)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, n ** dim))
    lhs, rhs = np.dot(A.apply(x), y), np.dot(x, A.apply(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    d = A.diagonal()
    e = np.zeros(n ** dim)
    for i in rng.integers(0, n ** dim, 5):
        e[:] = 0.0
        e[i] = 1.0
        assert A.apply(e)[i] == pytest.approx(d[i], rel=1e-14)
    assert np.all(d > 0)


def test_pointwise_loop_matches_vectorised_apply():
    p = gen.make_problem(3, 6, 3, 2.0, seed=2, convection=True)
    A = StencilOperator(3, 6, p.eta, p.vel)
    u = np.random.default_rng(1).standard_normal(A.N)
    full = A.apply(u)
    idx = np.arange(A.N)
    assert np.allclose(A.apply_at(u, idx), full, rtol=1e-13, atol=1e-13 * np.abs(full).max())


def test_convection_divergence_free_rows_and_transpose():
    n = 8
    p = gen.make_problem(3, n, 3, 2.0, seed=4, convection=True)
    Ad = StencilOperator(3, n, p.eta)
    Ac = StencilOperator(3, n, p.eta, p.vel)
    Ar = StencilOperator(3, n, p.eta, -p.vel)
    ones = np.ones(Ad.N)
    conv = (Ac.apply(ones) - Ad.apply(ones)).reshape(n, n, n)
    scale = np.abs(p.vel).max() * (n + 1)
    # interior rows (no boundary neighbour): net upwind flux of a constant = divergence = 0
    assert np.abs(conv[1:-1, 1:-1, 1:-1]).max() <= 1e-10 * scale
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal((2, Ad.N))
    cxy = np.dot(Ac.apply(x) - Ad.apply(x), y)
    xry = np.dot(x, Ar.apply(y) - Ad.apply(y))
    assert abs(cxy - xry) <= 1e-10 * scale * np.linalg.norm(x) * np.linalg.norm(y)


def test_divfree_velocity_scaling():
    n = 10
    g = np.random.default_rng(0)
    v = gen.divfree_face_velocity(n, g, cell_peclet=5.0)
    h = 1.0 / (n + 1)
    assert np.abs(v).max() * h / 2.0 == pytest.approx(5.0, rel=1e-12)
    div = (v[0][1:-1, 1:-1, 1:-1] - v[0][1:-1, 1:-1, :-2]
           + v[1][1:-1, 1:-1, 1:-1] - v[1][1:-1, :-2, 1:-1]
           + v[2][1:-1, 1:-1, 1:-1] - v[2][:-2, 1:-1, 1:-1])
    assert np.abs(div).max() <= 1e-12 * np.abs(v).max()


def test_sampled_apply_at_large_size():
    # the pointwise form is what GPU tests use to check sampled outputs at full size
    p = gen.make_problem(3, 20, 5, 4.0, seed=9)
    A = StencilOperator(3, 20, p.eta)
    u = np.random.default_rng(2).standard_normal(A.N)
    idx = np.random.default_rng(3).integers(0, A.N, 50)
    assert np.allclose(A.apply_at(u, idx), A.apply(u)[idx], rtol=1e-13)
