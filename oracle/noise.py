"""Counter-based Gaussian noise for the noisy preconditioner of section 2.2.1.

Test infrastructure (see the package docstring).

The toy study of section 2.2.1 (Figure 1) preconditions with B(r) = r plus
Gaussian noise of norm eta*||r||.  To compare a GPU solve with this oracle
draw for draw, both sides evaluate the same counter-based generator, each
from its published definition (nothing here is shared with the GPU code):

* Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4 x 64-bit counter and a 2 x 64-bit key; each
  of ten rounds multiplies counter words 0 and 2 by two fixed odd constants,
  keeps both halves of the 128-bit products and mixes the high halves with
  the other two counter words and the key; the key is advanced by two Weyl
  constants between rounds.
  Pin: numpy's own Philox bit generator (which increments its counter before
  each block), for arbitrary counters and keys.
* Box-Muller (Box and Muller, 1958): from two uniforms u1 in (0, 1] and
  u2 in [0, 1), g = sqrt(-2 ln u1) cos(2 pi u2) is standard normal.  The
  uniforms are the top 53 bits of Philox output words 0 and 1 (u1 offset by
  one unit so that it is never zero).  Only the cosine branch is used, one
  normal per counter.
  Pins: the closed form at hand-made words; sample moments and a
  Kolmogorov-Smirnov test against the normal law.

Element e of draw d under seed s takes counter (e, d, 0, 0) and key (s, 0).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)   # round multipliers
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)   # key increments (Weyl sequence)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.uint64, b: np.ndarray):
    """High and low 64-bit halves of the 128-bit products a*b (b an array)."""
    lo = a * b                                   # wraps mod 2^64
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64-10 of counters ``ctr`` (4 arrays or ints) under ``key`` (2).

    Returns the four output words as uint64 arrays.
    """
    with np.errstate(over="ignore"):
        c = [np.atleast_1d(np.asarray(v, dtype=np.uint64)).copy() for v in ctr]
        n = max(v.shape[0] for v in c)
        c = [np.broadcast_to(v, (n,)).copy() for v in c]
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        for rnd in range(10):
            if rnd:
                k0, k1 = k0 + _W0, k1 + _W1
            hi0, lo0 = _mulhilo(_M0, c[0])
            hi1, lo1 = _mulhilo(_M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def box_muller(w0: np.ndarray, w1: np.ndarray) -> np.ndarray:
    """Standard normals from two 64-bit words per sample (cosine branch)."""
    u1 = ((w0 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def gauss(seed: int, draw: int, n: int) -> np.ndarray:
    """n standard normals of draw ``draw`` under ``seed`` (element e: counter (e, draw, 0, 0))."""
    e = np.arange(n, dtype=np.uint64)
    w = philox4x64((e, np.uint64(draw), np.uint64(0), np.uint64(0)), (seed, 0))
    return box_muller(w[0], w[1])


class CounterNoisyPC:
    """B(r) = r + eta ||r|| g / ||g|| with g = gauss(seed, d, n) (section 2.2.1).

    d counts this object's earlier applications (0 for the first), so a solve
    that applies B in the algorithm's order sees draws 0, 1, 2, ...  A zero
    residual, or a zero noise vector, returns r unchanged.
    Pins: ||B(r) - r|| = eta ||r||; the Figure 1 behaviour (naive pipelining
    stagnates near eta, FCG and PIPEFCG converge) on the toy system.
    """

    def __init__(self, eta: float, seed: int):
        self.eta = float(eta)
        self.seed = int(seed)
        self.draws = 0

    def __call__(self, r: np.ndarray) -> np.ndarray:
        g = gauss(self.seed, self.draws, r.shape[0])
        self.draws += 1
        rn = float(np.linalg.norm(r))
        gn = float(np.linalg.norm(g))
        if rn == 0.0 or gn == 0.0:
            return r.copy()
        return r + self.eta * rn * g / gn
