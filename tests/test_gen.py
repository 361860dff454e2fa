"""Seeded input generators: the tensor-grid evaluation of the velocity
potential agrees with the pointwise definition, and draws are reproducible."""
import numpy as np

import gen


def test_potential_grid_evaluation_matches_pointwise():
    psi = gen._edge_potential(3, np.random.default_rng(5))
    xs, ys, zs = np.linspace(0, 1, 7), np.linspace(0, 1, 5) + 0.1, np.linspace(0, 1, 6) - 0.2
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    for c in range(3):
        assert np.abs(psi.grid(c, xs, ys, zs) - psi(c, X, Y, Z)).max() <= 1e-13


def test_problems_are_reproducible():
    a = gen.make_problem(3, 12, 3, 3.0, seed=4, convection=True)
    b = gen.make_problem(3, 12, 3, 3.0, seed=4, convection=True)
    assert np.array_equal(a.eta, b.eta) and np.array_equal(a.b, b.b) and np.array_equal(a.vel, b.vel)
