"""Flexible and pipelined flexible Krylov methods, FP64, plain numpy.

Test infrastructure (see the package docstring).

Each method follows its algorithm in the paper step by step (real
arithmetic, so conjugates and |beta|^2 become plain squares), with the
convergence test, truncation and restart handling that section 5 describes
and the listings omit.  Conventions shared with the GPU path:

* Iteration count = number of solution updates (CG/CR types) or Arnoldi
  columns (GMRES types).  Restarts do not reset it; everything counts toward
  ``maxit``.
* ``history[0]`` is ||b - A x0||_2; ``history[i]`` is the residual measure
  after iteration i: the recurred ||r_i||_2 for CG/CR types (its square is
  one more column of the same reduction), the Givens estimate |g_i| for
  GMRES types.
* Convergence: the first i with history[i] <= rtol*||b||_2.  The true
  residual ||b - A x|| is then checked; if it is above the tolerance the
  method restarts from x (a "gap" restart).
* Natural norm (section 5, implementation remarks: the one residual norm a
  pipelined CG/CR method has without an extra reduction): sqrt|gamma_i|,
  gamma = <u, r> for CG types and <r, A u> for CR types (u = B(r) or its
  recurrence).  ``natural[0]`` comes from the first start-up, ``natural[i]``
  from iteration i, whenever the method forms that gamma (FCG and GCR form
  it only after their 2-norm test, so the iteration that converges in the
  2-norm has none).  With ``norm="natural"`` the test is
  natural[i] <= rtol*natural[0], B is applied before the test, and the
  converged iterate is confirmed in the same norm of the true residual,
  sqrt|<B(r), r>| (CG) or sqrt|<r, A B(r)>| (CR) with r = b - A x, one more
  application of B ("other norms ... should be used to assess convergence",
  section 5); above the tolerance it is a gap restart.  If the first
  start-up already meets the 2-norm tolerance no natural tolerance exists
  and the 2-norm check decides.
  GMRES types have no natural norm and always test |g_i| (PCG, kept as
  FCG's pin, tests the 2-norm only).
* Window: the last nu_i directions, nu_i from ``truncation_nu`` with j the
  number of iterations since the last (re)start.
* Stagnation restart (option ``stall_window`` K, CG/CR types, 0 = off): once
  K iterations have passed since the (re)start, an iteration whose recurred
  residual is above half the one K iterations earlier restarts from x as a
  residual gap does (counted with the restarts).  Section 5's restarts flush
  the pipeline on a breakdown; a pipelined CG/CR method with an inexact B
  can instead stall at a noise floor that scales with ||A|| ||B|| (section
  2.2.1), and a restart from the current x rebuilds its recurrences there.
* Breakdown (section 5): eta_i <= 0 or non-finite for CG/CR types,
  t < 0 for PIPEFGMRES; restart from the current x, flushing the pipeline.
  A breakdown of the initial eta_0 is unrecoverable, as is exceeding
  ``max_restarts``.  ``force_breakdown_at`` (iteration index) triggers the
  breakdown branch for tests.

Readings of points the listings leave open (each restated where used):
PIPEFCG/PIPEGCR initialise m_0 = B(w_0), q_0 = B(s_0) as printed (exact for
linear B); PIPEGCR's initial gamma_0 = <r_0, s_0>, eta_0 = <s_0, s_0>
(the printed <r_0, A r_0> and ||s_0|| are inconsistent with its loop);
GCR takes alpha = <r, s>/<s, s> (minimal residual) with s recurred from
t = A u; PIPEFGMRES takes h_{j,i-1} for the printed h_{j,j-1}, wbar_0 =
A qbar_0, and the general z-bar update of its listing, which for constant
sigma is zbar_i = (wbar_{i-1} - sigma zbar_{i-1} - sum_j hbar_j zbar_j)/hbar.

Pins (tests/test_oracle_krylov.py): FCG and PIPEFCG with a fixed SPD
preconditioner and full window against scipy's CG residual history; GCR and
FGMRES with a fixed preconditioner against the minimum-residual solution over
the explicit Krylov space; PIPEGCR/PIPEFGMRES against GCR/FGMRES for linear
B; dense direct solves; A-conjugacy and Arnoldi invariants; Givens least
squares against numpy lstsq; the three-eigenvalue termination; and the
section 2.2.1 toy (naive pipelining stagnates near the noise level).
With a nonlinear B at workload sizes the exact iterates are parity unpinned
(no independent source exists); they are checked only through the invariants.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _dot(a, b) -> float:
    return float(np.dot(a, b))


def _norm(a) -> float:
    return math.sqrt(_dot(a, a))


def _finite_pos(v: float) -> bool:
    return math.isfinite(v) and v > 0.0


# ---------------------------------------------------------------------------
# Truncation rules (section 5, remark on truncation strategies)
# ---------------------------------------------------------------------------
def truncation_nu(rule: str, j: int, nu_max: int) -> int:
    """Number of previous directions used in the j-th iteration after a (re)start.

    'standard': min(j, nu_max).  'notay': max(1, j mod (nu_max+1)).
    'modp1': the authors' j mod nu_max + 1, capped at the j directions that
    exist (only p_0 exists at j = 1).
    """
    if j < 1:
        raise ValueError("j counts from 1")
    if rule == "standard":
        return min(j, nu_max)
    if rule == "notay":
        return max(1, j % (nu_max + 1))
    if rule == "modp1":
        return min(j, j % nu_max + 1)
    raise ValueError(rule)


# ---------------------------------------------------------------------------
# Givens least squares for the Hessenberg systems (section 4, on-the-fly QR)
# ---------------------------------------------------------------------------
class GivensLS:
    """Incremental QR of an upper Hessenberg matrix by Givens rotations.

    Column i (entries 0..i+1) is rotated by the previous rotations, a new
    rotation zeroes its subdiagonal, and the rotated right-hand side g
    (initially beta*e_0) gives the least-squares residual |g[i+1]|.
    """

    def __init__(self, m: int, beta: float):
        self.R = np.zeros((m + 1, m))
        self.c = np.zeros(m)
        self.s = np.zeros(m)
        self.g = np.zeros(m + 1)
        self.g[0] = beta
        self.ncol = 0

    def add_column(self, col: np.ndarray) -> float:
        i = self.ncol
        h = np.array(col[: i + 2], dtype=np.float64, copy=True)
        for j in range(i):
            a, b = h[j], h[j + 1]
            h[j] = self.c[j] * a + self.s[j] * b
            h[j + 1] = -self.s[j] * a + self.c[j] * b
        a, b = h[i], h[i + 1]
        d = math.hypot(a, b)
        if d == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / d, b / d
        self.c[i], self.s[i] = c, s
        h[i], h[i + 1] = d, 0.0
        self.R[: i + 2, i] = h
        gi = self.g[i]
        self.g[i] = c * gi
        self.g[i + 1] = -s * gi
        self.ncol = i + 1
        return abs(self.g[i + 1])

    def solve(self) -> np.ndarray:
        """Back substitution R y = g over the columns added so far."""
        k = self.ncol
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            acc = self.g[i]
            for j in range(i + 1, k):
                acc -= self.R[i, j] * y[j]
            y[i] = acc / self.R[i, i]
        return y


def givens_lstsq(H: np.ndarray, beta: float):
    """argmin_y ||beta e_0 - H y|| for (k+1) x k Hessenberg H; returns (y, residual)."""
    k = H.shape[1]
    G = GivensLS(k, beta)
    res = beta
    for i in range(k):
        res = G.add_column(H[:, i])
    return G.solve(), res


# ---------------------------------------------------------------------------
# Driver with restarts and the true-residual check
# ---------------------------------------------------------------------------
@dataclass
class Result:
    x: np.ndarray
    history: list
    iterations: int
    restarts: int
    converged: bool
    status: str                 # 'converged' | 'maxit' | 'breakdown'
    true_rel_resid: float
    trace: dict = field(default_factory=dict)
    natural: list = field(default_factory=list)


class _State:
    def __init__(self, maxit, force_breakdown_at, record, norm="2", rtol=0.0, stall_window=0):
        self.stall = stall_window
        self.it = 0
        self.history = []
        self.natural = []
        self.maxit = maxit
        self.force = force_breakdown_at
        self.record = record
        self.trace = {}
        self.norm = norm
        self.rtol = rtol
        self.ntol = 0.0

    @property
    def natural_test(self) -> bool:
        return self.norm == "natural"

    def start_natural(self, gamma):
        """natural[0] and the natural-norm tolerance, from the first start-up only."""
        if not self.natural:
            self.natural.append(math.sqrt(abs(gamma)))
            self.ntol = self.rtol * self.natural[0]

    def log_natural(self, gamma):
        self.natural.append(math.sqrt(abs(gamma)))

    def converged(self, tol) -> bool:
        """The convergence test of the chosen norm on the newest entries."""
        if self.natural_test:
            return self.natural[-1] <= self.ntol
        return self.history[-1] <= tol

    def stalled(self, j) -> bool:
        """Stagnation: at least ``stall`` iterations since the (re)start and the
        newest recurred residual above half the one ``stall`` iterations back."""
        return self.stall > 0 and j >= self.stall and self.history[-1] > 0.5 * self.history[-1 - self.stall]

    def forced(self, it=None) -> bool:
        """True once, at iteration ``force_breakdown_at`` (test hook)."""
        it = self.it if it is None else it
        if self.force >= 0 and it == self.force:
            self.force = -1
            return True
        return False


def solve(method: str, A, B, b, x0=None, rtol=1e-8, maxit=500, nu_max=30,
          truncation="standard", sigma=None, max_restarts=10,
          force_breakdown_at=-1, record=False, norm="2", stall_window=0) -> Result:
    """Solve A x = b with the named method.

    ``A`` is a callable (or an object with ``apply``), ``B`` a callable
    preconditioner.  ``nu_max`` is the window length for CG/CR types and the
    restart length m for GMRES types.  ``sigma`` is PIPEFGMRES's constant
    shift (default: ``estimate_sigma``).  ``norm`` is "2" or "natural" (the
    convergence measure of CG/CR types, see the module docstring).
    """
    if norm not in ("2", "natural"):
        raise ValueError("norm must be '2' or 'natural'")
    Aop = A.apply if hasattr(A, "apply") else A
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = _norm(b)
    if bnorm == 0.0:
        return Result(np.zeros_like(b), [0.0], 0, 0, True, "converged", 0.0)
    tol = rtol * bnorm
    cycle = METHODS[method]
    kw = dict(nu_max=nu_max, trunc=truncation)
    if method == "pipefgmres":
        kw["sigma"] = estimate_sigma(Aop, B, b.shape[0]) if sigma is None else float(sigma)
    no_natural = method in ("pcg", "fgmres", "pipefgmres")
    st = _State(maxit, force_breakdown_at, record, "2" if no_natural else norm, rtol,
                0 if method in ("pcg", "fgmres", "pipefgmres") else stall_window)
    restarts = 0
    status = "maxit"
    cr = method in _CR_TYPES
    while True:
        reason = cycle(Aop, B, b, x, st, tol, **kw)
        if reason == "converged":
            if st.natural_test and st.natural:
                ok = _true_natural(Aop, B, b, x, cr) <= st.ntol
            else:
                ok = _norm(b - Aop(x)) <= tol
            if ok:
                status = "converged"
                break
            reason = "gap"
        if reason == "maxit":
            status = "maxit"
            break
        if reason == "breakdown0":
            status = "breakdown"
            break
        if reason in ("breakdown", "gap"):
            restarts += 1
            if restarts > max_restarts:
                status = "breakdown" if reason == "breakdown" else "maxit"
                break
        # 'cycle' (GMRES restart), 'breakdown' and 'gap' continue from x
        if st.it >= maxit:
            status = "maxit"
            break
    true_rel = _norm(b - Aop(x)) / bnorm
    return Result(x, st.history, st.it, restarts, status == "converged", status, true_rel, st.trace,
                  st.natural)


_CR_TYPES = ("gcr", "pipegcr", "pipegcr_w", "pipegcr_naive", "pipegcr_w_naive")


def _true_natural(Aop, B, b, x, cr):
    """The natural norm of the true residual r = b - A x: sqrt|<B(r), r>| for
    CG types, sqrt|<r, A B(r)>| for CR types (one more application of B).
    Section 5 advises checking convergence in other norms as well; a
    natural-norm test on the recurred quantities is confirmed with it."""
    r = b - Aop(x)
    u = B(r)
    g = _dot(r, Aop(u)) if cr else _dot(u, r)
    return math.sqrt(abs(g))


def _start(Aop, b, x, st, tol):
    """r = b - A x; record history[0] once; report whether x already converged."""
    r = b - Aop(x)
    rn = _norm(r)
    if not st.history:
        st.history.append(rn)
    return r, rn <= tol


def _window(P, nu):
    return range(len(P) - nu, len(P))


# ---------------------------------------------------------------------------
# CG family
# ---------------------------------------------------------------------------
def _pcg_cycle(Aop, B, b, x, st, tol, nu_max, trunc):
    """Preconditioned CG (Alg. 3) with a linear B = M^-1."""
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    u = B(r)
    p = u.copy()
    s = Aop(p)
    gamma = _dot(u, r)
    eta = _dot(s, p)
    if not _finite_pos(eta):
        return "breakdown0"
    alpha = gamma / eta
    while True:
        if st.it >= st.maxit:
            return "maxit"
        st.it += 1
        x += alpha * p
        r -= alpha * s
        st.history.append(_norm(r))
        if st.history[-1] <= tol:
            return "converged"
        u = B(r)
        gamma_new = _dot(u, r)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = u + beta * p
        s = Aop(p)
        eta = _dot(s, p)
        if st.forced() or not _finite_pos(eta):
            return "breakdown"
        alpha = gamma / eta


def _fcg_cycle(Aop, B, b, x, st, tol, nu_max, trunc):
    """Flexible CG (Alg. 2): two reductions per iteration."""
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    u = B(r)
    P = [u.copy()]
    S = [Aop(P[0])]
    gamma = _dot(u, r)
    st.start_natural(gamma)
    ETA = [_dot(P[0], S[0])]
    if not _finite_pos(ETA[0]):
        return "breakdown0"
    alpha = gamma / ETA[0]
    j = 0
    while True:
        if st.it >= st.maxit:
            return "maxit"
        st.it += 1
        j += 1
        x += alpha * P[-1]
        r -= alpha * S[-1]
        st.history.append(_norm(r))
        if not st.natural_test and st.converged(tol):
            return "converged"
        if not st.natural_test and st.stalled(j):
            return "gap"
        u = B(r)
        gamma = _dot(u, r)
        st.log_natural(gamma)
        if st.natural_test and st.converged(tol):
            return "converged"
        if st.natural_test and st.stalled(j):
            return "gap"
        nu = truncation_nu(trunc, j, nu_max)
        win = _window(P, nu)
        beta = {k: -_dot(u, S[k]) / ETA[k] for k in win}
        p = u.copy()
        for k in win:
            p += beta[k] * P[k]
        s = Aop(p)
        eta = _dot(p, s)
        if st.forced() or not _finite_pos(eta):
            return "breakdown"
        alpha = gamma / eta
        P.append(p)
        S.append(s)
        ETA.append(eta)
        if len(P) > nu_max:
            del P[0], S[0], ETA[0]
        if st.record:
            st.trace.setdefault("P", []).append(p.copy())


def _pipefcg_cycle(Aop, B, b, x, st, tol, nu_max, trunc, naive=False):
    """PIPEFCG (Alg. 8); with ``naive`` the unstabilised m_i = B(w_i) of Alg. 7.

    One reduction per iteration (gamma, delta, the window dots and <r, r>);
    in a parallel code it overlaps the preconditioner and operator applies
    that follow it.  m_0 = B(w_0) as printed in the initialisation.
    """
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    u = B(r)
    w = Aop(u)
    m = B(w)
    n = Aop(m)
    gamma = _dot(u, r)
    delta = _dot(u, w)
    st.start_natural(gamma)
    P, S, Q, Z = [u.copy()], [w.copy()], [m.copy()], [n.copy()]
    ETA = [delta]
    if not _finite_pos(delta):
        return "breakdown0"
    alpha = gamma / delta
    j = 0
    while True:
        if st.it >= st.maxit:
            return "maxit"
        st.it += 1
        j += 1
        x += alpha * P[-1]
        r -= alpha * S[-1]
        u -= alpha * Q[-1]
        w -= alpha * Z[-1]
        nu = truncation_nu(trunc, j, nu_max)
        win = _window(P, nu)
        # the single reduction
        gamma = _dot(u, r)
        delta = _dot(u, w)
        dks = {k: _dot(u, S[k]) for k in win}
        rho = _dot(r, r)
        st.history.append(math.sqrt(rho))
        st.log_natural(gamma)
        if st.converged(tol):
            return "converged"
        if st.stalled(j):
            return "gap"
        # overlapped with the reduction
        m = B(w) if naive else u + B(w - r)
        n = Aop(m)
        beta = {k: -dks[k] / ETA[k] for k in win}
        p, s, q, z = u.copy(), w.copy(), m.copy(), n.copy()
        for k in win:
            p += beta[k] * P[k]
            s += beta[k] * S[k]
            q += beta[k] * Q[k]
            z += beta[k] * Z[k]
        eta = delta - sum(beta[k] * beta[k] * ETA[k] for k in win)
        if st.forced() or not _finite_pos(eta):
            return "breakdown"
        alpha = gamma / eta
        for L, v in ((P, p), (S, s), (Q, q), (Z, z)):
            L.append(v)
        ETA.append(eta)
        if len(P) > nu_max:
            for L in (P, S, Q, Z, ETA):
                del L[0]
        if st.record:
            st.trace.setdefault("P", []).append(p.copy())
            st.trace.setdefault("S", []).append(s.copy())


def _naive_pipefcg_cycle(*a, **k):
    return _pipefcg_cycle(*a, naive=True, **k)


# ---------------------------------------------------------------------------
# CR family
# ---------------------------------------------------------------------------
def _gcr_cycle(Aop, B, b, x, st, tol, nu_max, trunc):
    """Generalized CR (Alg. 9), minimal-residual alpha = <r,s>/<s,s>.

    Alg. 9 needs <A u_i, s_k>; t = A u is formed once and s_i is recurred as
    t + sum beta s_k (equal to A p_i by linearity), one operator apply per
    iteration.  Two reductions: the window dots, then <r,s> and <s,s>.
    """
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    u = B(r)
    P = [u.copy()]
    S = [Aop(P[0])]
    gamma = _dot(r, S[0])
    st.start_natural(gamma)
    ETA = [_dot(S[0], S[0])]
    if not _finite_pos(ETA[0]):
        return "breakdown0"
    alpha = gamma / ETA[0]
    j = 0
    while True:
        if st.it >= st.maxit:
            return "maxit"
        st.it += 1
        j += 1
        x += alpha * P[-1]
        r -= alpha * S[-1]
        st.history.append(_norm(r))
        if not st.natural_test and st.converged(tol):
            return "converged"
        if not st.natural_test and st.stalled(j):
            return "gap"
        u = B(r)
        t = Aop(u)
        st.log_natural(_dot(r, t))
        if st.natural_test and st.converged(tol):
            return "converged"
        if st.natural_test and st.stalled(j):
            return "gap"
        nu = truncation_nu(trunc, j, nu_max)
        win = _window(P, nu)
        beta = {k: -_dot(t, S[k]) / ETA[k] for k in win}
        p, s = u.copy(), t.copy()
        for k in win:
            p += beta[k] * P[k]
            s += beta[k] * S[k]
        gamma = _dot(r, s)
        eta = _dot(s, s)
        if st.forced() or not _finite_pos(eta):
            return "breakdown"
        alpha = gamma / eta
        P.append(p)
        S.append(s)
        ETA.append(eta)
        if len(P) > nu_max:
            del P[0], S[0], ETA[0]


def _pipegcr_cycle(Aop, B, b, x, st, tol, nu_max, trunc, recur_w=False, naive=False):
    """PIPEGCR (Alg. 11); with ``recur_w`` PIPEGCR_w (Alg. 12).

    Initialisation reads gamma_0 = <r_0, s_0>, eta_0 = <s_0, s_0>, q_0 = B(s_0)
    (and z_0 = A q_0, w_0 = s_0 for the recurred-w variant); the tilde-u of
    the listing is the recurred u throughout.

    ``naive`` replaces the stabilised m_i = u_i + B(w_i - r_i) of section
    2.2.2 by m_i = B(w_i), the CR counterpart of the naive pipelining that
    Alg. 7 shows for FCG (identical for linear B).  It exists so a test can
    show that the stabilised form is the one written here: with a noisy B
    the naive cycle stalls near the noise level while PIPEGCR converges.
    Pinned by that contrast (tests/test_oracle_krylov.py).
    """
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    u = B(r)
    P = [u.copy()]
    S = [Aop(P[0])]
    Q = [B(S[0])]
    Zw = [Aop(Q[0])] if recur_w else None
    w = S[0].copy() if recur_w else None
    gamma = _dot(r, S[0])
    st.start_natural(gamma)
    ETA = [_dot(S[0], S[0])]
    if not _finite_pos(ETA[0]):
        return "breakdown0"
    alpha = gamma / ETA[0]
    j = 0
    while True:
        if st.it >= st.maxit:
            return "maxit"
        st.it += 1
        j += 1
        x += alpha * P[-1]
        r -= alpha * S[-1]
        u -= alpha * Q[-1]
        if recur_w:
            w -= alpha * Zw[-1]
        else:
            w = Aop(u)
        nu = truncation_nu(trunc, j, nu_max)
        win = _window(P, nu)
        gamma = _dot(r, w)
        delta = _dot(w, w)
        dks = {k: _dot(w, S[k]) for k in win}
        rho = _dot(r, r)
        st.history.append(math.sqrt(rho))
        st.log_natural(gamma)
        if st.converged(tol):
            return "converged"
        if st.stalled(j):
            return "gap"
        m = B(w) if naive else u + B(w - r)
        nn = Aop(m) if recur_w else None
        beta = {k: -dks[k] / ETA[k] for k in win}
        p, s, q = u.copy(), w.copy(), m.copy()
        z = nn.copy() if recur_w else None
        for k in win:
            p += beta[k] * P[k]
            s += beta[k] * S[k]
            q += beta[k] * Q[k]
            if recur_w:
                z += beta[k] * Zw[k]
        eta = delta - sum(beta[k] * beta[k] * ETA[k] for k in win)
        if st.forced() or not _finite_pos(eta):
            return "breakdown"
        alpha = gamma / eta
        P.append(p)
        S.append(s)
        Q.append(q)
        ETA.append(eta)
        if recur_w:
            Zw.append(z)
        if len(P) > nu_max:
            for L in (P, S, Q, ETA) + ((Zw,) if recur_w else ()):
                del L[0]


def _pipegcr_w_cycle(*a, **k):
    return _pipegcr_cycle(*a, recur_w=True, **k)


def _naive_pipegcr_cycle(*a, **k):
    return _pipegcr_cycle(*a, naive=True, **k)


def _naive_pipegcr_w_cycle(*a, **k):
    return _pipegcr_cycle(*a, recur_w=True, naive=True, **k)


# ---------------------------------------------------------------------------
# GMRES family
# ---------------------------------------------------------------------------
def _fgmres_cycle(Aop, B, b, x, st, tol, nu_max, trunc):
    """One restart cycle of FGMRES (Alg. 13): CGS Arnoldi, two reductions per column."""
    m = nu_max
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    beta0 = _norm(r)
    Pb = [r / beta0]
    U = [B(Pb[0])]
    z = Aop(U[0])
    G = GivensLS(m, beta0)
    H = np.zeros((m + 1, m))
    for i in range(1, m + 1):
        if st.it >= st.maxit:
            _fgmres_update(x, U, G)
            return "maxit"
        for j in range(i):
            H[j, i - 1] = _dot(Pb[j], z)
        pbar = z.copy()
        for j in range(i):
            pbar -= H[j, i - 1] * Pb[j]
        hn = _norm(pbar)
        H[i, i - 1] = hn
        st.it += 1
        res = G.add_column(H[:, i - 1])
        st.history.append(res)
        if st.record:
            st.trace["H"] = H[: i + 1, :i].copy()
            st.trace["P"] = [v.copy() for v in Pb]
            st.trace["U"] = [v.copy() for v in U]
        if res <= tol or hn == 0.0:
            _fgmres_update(x, U, G)
            return "converged"
        if i == m:
            _fgmres_update(x, U, G)
            return "cycle"
        Pb.append(pbar / hn)
        U.append(B(Pb[i]))
        z = Aop(U[i])
    return "cycle"


def _fgmres_update(x, U, G):
    if G.ncol == 0:
        return
    y = G.solve()
    for j in range(G.ncol):
        x += y[j] * U[j]


def _pipefgmres_cycle(Aop, B, b, x, st, tol, nu_max, trunc, sigma):
    """One restart cycle of PIPEFGMRES (Alg. 15) with a constant shift sigma.

    One reduction per column (the window dots and ||zbar||^2); the norm of the
    new basis vector comes from t = ||zbar||^2 - sum hbar^2; t < 0 is a norm
    breakdown (least squares over the finished columns, then restart).
    """
    m = nu_max
    r, done = _start(Aop, b, x, st, tol)
    if done:
        return "converged"
    beta0 = _norm(r)
    Pb = [r / beta0]
    U = [B(Pb[0])]
    ZB = [Aop(U[0]) - sigma * Pb[0]]
    qb = B(ZB[0])
    wb = Aop(qb)
    G = GivensLS(m, beta0)
    H = np.zeros((m + 1, m))
    for i in range(1, m + 1):
        if st.it >= st.maxit:
            _fgmres_update(x, U, G)
            return "maxit"
        z = ZB[i - 1]
        hb = np.array([_dot(Pb[j], z) for j in range(i)])
        zeta = _dot(z, z)
        t = zeta - float(np.sum(hb * hb))
        if st.forced(st.it + 1) or t < 0.0:
            _fgmres_update(x, U, G)
            return "breakdown"
        H[:i, i - 1] = hb
        H[i - 1, i - 1] += sigma
        hn = math.sqrt(t)
        H[i, i - 1] = hn
        st.it += 1
        res = G.add_column(H[:, i - 1])
        st.history.append(res)
        if st.record:
            st.trace["H"] = H[: i + 1, :i].copy()
            st.trace["P"] = [v.copy() for v in Pb]
            st.trace["U"] = [v.copy() for v in U]
            st.trace["ZB"] = [v.copy() for v in ZB]
        if res <= tol or hn == 0.0:
            _fgmres_update(x, U, G)
            return "converged"
        if i == m:
            _fgmres_update(x, U, G)
            return "cycle"
        p_new = z.copy()
        u_new = qb.copy()
        z_new = wb - sigma * z
        for j in range(i):
            p_new -= hb[j] * Pb[j]
            u_new -= hb[j] * U[j]
            z_new -= hb[j] * ZB[j]
        Pb.append(p_new / hn)
        U.append(u_new / hn)
        ZB.append(z_new / hn)
        qb = B(ZB[i])
        wb = Aop(qb)
    return "cycle"


def estimate_sigma(Aop, B, N: int, its: int = 10) -> float:
    """PIPEFGMRES shift: Rayleigh quotient of v -> A B(v) after ``its`` power steps.

    The paper sets sigma to a constant approximating the largest eigenvalue
    of the (right-)preconditioned operator (sections 4.4 and 5); the start
    vector is the normalised all-ones vector.  The parity tests of the
    methods pass sigma explicitly.

    Pins (tests/test_oracle_krylov.py): for diagonal A and B the estimate is
    the closed form sum(mu^(2k-1)) / sum(mu^(2k-2)) over the eigenvalues mu
    of A B (k = its, equal start weights), it approaches max(mu) within the
    power-iteration bound, and on a small stencil operator with Jacobi B it
    converges to the largest eigenvalue of A D^-1 from a dense solver.
    """
    v = np.ones(N) / math.sqrt(N)
    lam = 0.0
    for _ in range(its):
        w = Aop(B(v))
        lam = _dot(v, w)
        nw = _norm(w)
        if nw == 0.0:
            break
        v = w / nw
    return lam


METHODS = {
    "pcg": _pcg_cycle,
    "fcg": _fcg_cycle,
    "pipefcg": _pipefcg_cycle,
    "pipefcg_naive": _naive_pipefcg_cycle,
    "gcr": _gcr_cycle,
    "pipegcr": _pipegcr_cycle,
    "pipegcr_w": _pipegcr_w_cycle,
    "pipegcr_naive": _naive_pipegcr_cycle,
    "pipegcr_w_naive": _naive_pipegcr_w_cycle,
    "fgmres": _fgmres_cycle,
    "pipefgmres": _pipefgmres_cycle,
}
