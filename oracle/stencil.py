"""Variable-coefficient finite-difference operators, FP64, plain numpy.

Test infrastructure (see the package docstring).

The operator is the 2nd-order finite-difference stencil the paper's
performance model assumes for SpMV (section 7: nz = 7 nonzeros per row in 3D,
5 in 2D), applied to -div(eta grad u) [+ div(v u)] on the unit box with
homogeneous Dirichlet boundaries:

    (A u)_i = h^-2 * sum_f k_f (u_i - u_nb(f))
            + h^-1 * sum_f ( max(v_f, 0) u_i + min(v_f, 0) u_nb(f) )

over the 2*dim faces f of node i, where u_nb = 0 on the boundary, k_f is the
harmonic mean of eta at the two nodes of the face and v_f is the outward
face-normal velocity (first-order upwind flux).  Vectors cover interior nodes
only, x fastest; ``eta`` and the face velocities live on the padded grid
(see ``gen``).

Parity pins (tests/test_oracle_stencil.py): eta = 1 reduces to the textbook
Laplacian assembled from 1D second differences with scipy.sparse and has the
closed-form sine eigenpairs; symmetry of the diffusion part; an entry-by-entry
pure-Python loop on tiny grids; zero interior row sums of the convection part
for a discretely divergence-free field and transposition under v -> -v.
"""
from __future__ import annotations

import numpy as np


def harmonic_face(a, b):
    """Face coefficient: harmonic mean 2ab/(a+b) of the two node viscosities."""
    return 2.0 * a * b / (a + b)


class StencilOperator:
    """A = -div(eta grad .) [+ upwind div(v .)] on n^dim interior nodes."""

    def __init__(self, dim: int, n: int, eta: np.ndarray, vel: np.ndarray | None = None):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if eta.shape != (n + 2,) * dim:
            raise ValueError("eta must be on the padded grid")
        if vel is not None and (dim != 3 or vel.shape != (3,) + (n + 2,) * 3):
            raise ValueError("face velocities are (3, n+2, n+2, n+2)")
        self.dim, self.n = dim, n
        self.h = 1.0 / (n + 1)
        self.eta = np.asarray(eta, dtype=np.float64)
        self.vel = None if vel is None else np.asarray(vel, dtype=np.float64)

    @property
    def N(self) -> int:
        return self.n ** self.dim

    # -- index helpers ------------------------------------------------------
    def _sl(self, axis: int, shift: int):
        """Padded-grid slice of interior nodes shifted by ``shift`` along numpy axis ``axis``."""
        n = self.n
        s = [slice(1, n + 1)] * self.dim
        s[axis] = slice(1 + shift, n + 1 + shift)
        return tuple(s)

    def _faces(self):
        """Yield (numpy axis, coordinate c, sign) for the 2*dim faces (x, y, z order)."""
        for c in range(self.dim):
            axis = self.dim - 1 - c          # arrays are [z][y][x]
            for sgn in (+1, -1):
                yield axis, c, sgn

    def _outward_velocity(self, c: int, sgn: int, axis: int):
        """Outward normal velocity on the (c, sgn) face of every interior node."""
        if sgn > 0:
            return self.vel[c][self._sl(axis, 0)]
        return -self.vel[c][self._sl(axis, -1)]

    # -- operator -----------------------------------------------------------
    def apply(self, u: np.ndarray) -> np.ndarray:
        n, dim, h = self.n, self.dim, self.h
        U = np.zeros((n + 2,) * dim)
        U[(slice(1, n + 1),) * dim] = np.asarray(u, dtype=np.float64).reshape((n,) * dim)
        c0 = (slice(1, n + 1),) * dim
        uc = U[c0]
        ec = self.eta[c0]
        y = np.zeros((n,) * dim)
        for axis, c, sgn in self._faces():
            nb = self._sl(axis, sgn)
            k = harmonic_face(ec, self.eta[nb])
            y += k * (uc - U[nb]) / (h * h)
        if self.vel is not None:
            for axis, c, sgn in self._faces():
                nb = self._sl(axis, sgn)
                vn = self._outward_velocity(c, sgn, axis)
                y += (np.maximum(vn, 0.0) * uc + np.minimum(vn, 0.0) * U[nb]) / h
        return y.reshape(-1)

    __call__ = apply

    def diagonal(self) -> np.ndarray:
        """diag(A): h^-2 sum_f k_f (+ h^-1 sum_f max(v_f, 0))."""
        n, dim, h = self.n, self.dim, self.h
        c0 = (slice(1, n + 1),) * dim
        ec = self.eta[c0]
        d = np.zeros((n,) * dim)
        for axis, c, sgn in self._faces():
            d += harmonic_face(ec, self.eta[self._sl(axis, sgn)]) / (h * h)
        if self.vel is not None:
            for axis, c, sgn in self._faces():
                d += np.maximum(self._outward_velocity(c, sgn, axis), 0.0) / h
        return d.reshape(-1)

    def apply_at(self, u: np.ndarray, idx) -> np.ndarray:
        """(A u) at selected flat interior indices only, one node at a time.

        Used to check sampled outputs at sizes where a full apply is not wanted.
        """
        n, dim, h = self.n, self.dim, self.h
        uu = np.asarray(u, dtype=np.float64).reshape((n,) * dim)
        out = np.empty(len(idx))
        for t, flat in enumerate(np.asarray(idx, dtype=np.int64)):
            ii = list(np.unravel_index(int(flat), (n,) * dim))   # [z][y][x] interior
            pc = tuple(a + 1 for a in ii)                         # padded index
            val = 0.0
            for axis, c, sgn in self._faces():
                pn = list(pc)
                pn[axis] += sgn
                inside = 1 <= pn[axis] <= n
                unb = uu[tuple(a - 1 for a in pn)] if inside else 0.0
                k = harmonic_face(self.eta[pc], self.eta[tuple(pn)])
                val += k * (uu[tuple(ii)] - unb) / (h * h)
                if self.vel is not None:
                    if sgn > 0:
                        vn = self.vel[c][pc]
                    else:
                        vn = -self.vel[c][tuple(pn)]
                    val += (max(vn, 0.0) * uu[tuple(ii)] + min(vn, 0.0) * unb) / h
            out[t] = val
        return out
