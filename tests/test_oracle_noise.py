"""Pins for the oracle's counter-based noise and seeded noisy preconditioner (CPU only).

Independent references: numpy's Philox bit generator (a library
implementation of the same published generator), the Box-Muller closed form
at hand-made words, the normal law (moments, Kolmogorov-Smirnov), the noisy
preconditioner's norm identity and the section 2.2.1 toy study (Figure 1).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import gen
from oracle import CounterNoisyPC, box_muller, gauss, philox4x64, solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASK64 = (1 << 64) - 1


def _numpy_philox_block(ctr, key):
    """numpy's Philox4x64-10 at counter ``ctr``: it increments before each block."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & MASK64 for i in range(4)]
    bg = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                          key=np.array([int(key[0]), int(key[1])], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((0, 7, 0, 0), (12345, 0)),                       # element 0 of draw 7: the decrement borrows
    ((123456789, 3, 0, 0), (2 ** 63 + 5, 0)),
    ((MASK64, MASK64, MASK64, MASK64), (MASK64, MASK64)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(ctr, key):
    mine = [int(w[0]) for w in philox4x64(ctr, key)]
    assert mine == _numpy_philox_block(ctr, key)


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(4)
    e = rng.integers(0, 2 ** 63, size=64, dtype=np.uint64)
    out = philox4x64((e, np.uint64(9), np.uint64(0), np.uint64(0)), (77, 0))
    for i in (0, 5, 63):
        ref = _numpy_philox_block((int(e[i]), 9, 0, 0), (77, 0))
        assert [int(w[i]) for w in out] == ref


def test_box_muller_closed_form():
    half = np.uint64(((1 << 52) - 1) << 11)          # u1 = 1/2
    w1 = np.array([0, (1 << 51) << 11, (1 << 52) << 11], dtype=np.uint64)   # u2 = 0, 1/4, 1/2
    g = box_muller(np.full(3, half, dtype=np.uint64), w1)
    r = math.sqrt(2.0 * math.log(2.0))
    assert g[0] == pytest.approx(r, rel=1e-15)
    assert abs(g[1]) < 1e-15
    assert g[2] == pytest.approx(-r, rel=1e-15)
    # u1 = 1 (all top bits set) gives exactly zero; u1 = 2^-53 the largest radius
    top = np.array([MASK64, 0], dtype=np.uint64)
    g = box_muller(top, np.zeros(2, dtype=np.uint64))
    assert g[0] == 0.0
    assert g[1] == pytest.approx(math.sqrt(2.0 * 53 * math.log(2.0)), rel=1e-15)


def test_gauss_is_standard_normal():
    n = 200_000
    g = gauss(2024, 0, n)
    assert abs(g.mean()) < 5.0 / math.sqrt(n)
    assert abs(g.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
    assert abs(scipy.stats.skew(g)) < 5.0 * math.sqrt(6.0 / n)
    assert abs(scipy.stats.kurtosis(g)) < 5.0 * math.sqrt(24.0 / n)
    assert scipy.stats.kstest(g, "norm").pvalue > 1e-4
    # draws and seeds give independent streams
    h = gauss(2024, 1, n)
    k = gauss(2025, 0, n)
    assert abs(np.corrcoef(g, h)[0, 1]) < 5.0 / math.sqrt(n)
    assert abs(np.corrcoef(g, k)[0, 1]) < 5.0 / math.sqrt(n)
    # element e does not depend on n
    np.testing.assert_array_equal(gauss(2024, 0, 1000), g[:1000])


def test_counter_noisy_pc_definition():
    rng = np.random.default_rng(0)
    r = rng.standard_normal(500)
    for eta in (0.1, 1e-3):
        B = CounterNoisyPC(eta, 11)
        y0 = B(r)
        y1 = B(r)
        assert B.draws == 2
        assert np.linalg.norm(y0 - r) == pytest.approx(eta * np.linalg.norm(r), rel=1e-13)
        assert not np.array_equal(y0, y1)                      # a fresh draw per application
        g = gauss(11, 0, r.shape[0])
        # y0 - r cancels: its rounding error is relative to |r|, not to the noise
        np.testing.assert_allclose(y0 - r, eta * np.linalg.norm(r) * g / np.linalg.norm(g),
                                   rtol=1e-12, atol=4e-16 * np.abs(r).max())
        assert np.array_equal(CounterNoisyPC(eta, 11)(r), y0)  # reproducible
    B = CounterNoisyPC(0.1, 3)
    assert np.array_equal(B(np.zeros(7)), np.zeros(7))
    assert B.draws == 1


def test_fig1_toy_with_counter_noise():
    """Figure 1 (section 2.2.1) with the seeded counter-based noise."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_toy.json")))
    lam, b = gen.toy_diagonal(g["problem"]["n"], g["problem"]["condition_number"])
    xs = b / lam
    lo, hi = g["plateau_band"]
    for eta in g["noise_levels"]:
        err = {}
        for m in ("fcg", "pipefcg_naive", "pipefcg"):
            B = CounterNoisyPC(eta, 5)
            r = solve(m, lambda v: lam * v, B, b, rtol=1e-15, maxit=g["check_at_iteration"], nu_max=g["nu_max"])
            err[m] = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
        assert lo * eta <= err["pipefcg_naive"] <= hi * eta, (eta, err)
        assert err["fcg"] < g["converged_error_below"] and err["pipefcg"] < g["converged_error_below"], err
