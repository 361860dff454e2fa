"""Pins for the oracle's Krylov methods (CPU only).

Independent references: scipy's CG, least squares over an explicitly built
Krylov basis, dense direct solves, numpy lstsq, closed-form termination, the
paper's toy stagnation study and the algebraic invariants of each method.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import gen
from oracle import (StencilOperator, givens_lstsq, jacobi_pc, make_pc, noisy_pc,
                    solve, truncation_nu)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(dim=2, n=8, contrast=2.0, seed=0, conv=False):
    p = gen.make_problem(dim, n, 2, contrast, seed, convection=conv)
    return StencilOperator(dim, n, p.eta, p.vel), p.b


def _dense(A):
    return np.array([A.apply(e) for e in np.eye(A.N)]).T


def _scipy_cg_history(A, b, Dinv, its):
    hist = [np.linalg.norm(b)]
    L = spla.LinearOperator((A.N, A.N), matvec=A.apply, dtype=np.float64)
    M = spla.LinearOperator((A.N, A.N), matvec=lambda t: Dinv * t, dtype=np.float64)
    spla.cg(L, b, x0=np.zeros(A.N), rtol=0.0, atol=0.0, maxiter=its, M=M,
            callback=lambda xk: hist.append(np.linalg.norm(b - A.apply(xk))))
    return np.array(hist)


def _min_residual_history(A, b, Minv, its):
    """min ||b - A x|| over x in K_i(M^-1 A, M^-1 b), i = 1..its, by lstsq."""
    V = [Minv(b)]
    V[0] = V[0] / np.linalg.norm(V[0])
    out = [np.linalg.norm(b)]
    for i in range(1, its + 1):
        Vm = np.array(V).T
        AV = np.array([A.apply(v) for v in V]).T
        c = np.linalg.lstsq(AV, b, rcond=None)[0]
        out.append(np.linalg.norm(b - AV @ c))
        t = Minv(A.apply(V[-1]))
        V.append(t / np.linalg.norm(t))
    return np.array(out)


# --- CG family -------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 12])
@pytest.mark.parametrize("method", ["fcg", "pcg"])
def test_fcg_full_window_reproduces_pcg(n, method):
    A, b = _tiny(2, n, 2.0)
    Dinv = 1.0 / A.diagonal()
    its = 18 if n == 8 else 25
    ref = _scipy_cg_history(A, b, Dinv, its)
    r = solve(method, A, jacobi_pc(Dinv), b, rtol=1e-13, maxit=its, nu_max=its)
    h = np.array(r.history)
    k = min(len(h), len(ref))
    keep = ref[:k] > 1e-9 * ref[0]
    assert np.allclose(h[:k][keep], ref[:k][keep], rtol=1e-10, atol=0)


def test_pipefcg_linear_pc_matches_cg_early():
    A, b = _tiny(2, 10, 1.0, seed=2)
    Dinv = 1.0 / A.diagonal()
    ref = _scipy_cg_history(A, b, Dinv, 10)
    r = solve("pipefcg", A, jacobi_pc(Dinv), b, rtol=1e-14, maxit=10, nu_max=30)
    assert np.allclose(np.array(r.history)[:11], ref[:11], rtol=1e-8)


def test_three_eigenvalues_terminate_in_three_steps():
    lam = np.repeat([1.0, 2.0, 5.0], 10)
    b = np.random.default_rng(0).standard_normal(30)
    for method in ("fcg", "pipefcg", "gcr", "pipegcr"):
        r = solve(method, lambda v: lam * v, lambda v: v.copy(), b, rtol=1e-12, maxit=10, nu_max=5)
        assert r.converged and r.iterations == 3, (method, r.iterations, r.history)


@pytest.mark.parametrize("method,pc", [("fcg", "jacobi_pcg"), ("gcr", "jacobi_pcg"),
                                       ("fgmres", "jacobi_pcg"), ("pipefgmres", "jacobi_pcg"),
                                       ("pipefcg", "jacobi"), ("pipegcr", "jacobi")])
def test_final_answer_matches_dense_solve(method, pc):
    # pipelined CG/CR types need a faithful preconditioner (section 2.2.2);
    # the global few-step inner CG is not one at this contrast, so they get Jacobi
    A, b = _tiny(2, 8, 2.0, seed=4)
    xs = np.linalg.solve(_dense(A), b)
    r = solve(method, A, make_pc(pc, A, 2), b, rtol=1e-11, maxit=400, nu_max=30, sigma=None)
    assert r.converged, (method, r.status, r.history[-3:])
    assert r.true_rel_resid <= 1e-11
    kappa = np.linalg.cond(_dense(A))
    assert np.linalg.norm(r.x - xs) <= kappa * 1e-11 * np.linalg.norm(xs)


def test_conjugacy_and_recurrences_with_nonlinear_pc():
    A, b = _tiny(2, 12, 2.0, seed=5)
    B = make_pc("jacobi_pcg", A, 2)
    for method in ("fcg", "pipefcg"):
        r = solve(method, A, B, b, rtol=1e-14, maxit=8, nu_max=30, record=True)
        P = r.trace["P"]
        AP = [A.apply(p) for p in P]
        for i in range(len(P)):
            for k in range(i):
                c = abs(np.dot(P[i], AP[k])) / math.sqrt(np.dot(P[i], AP[i]) * np.dot(P[k], AP[k]))
                assert c < 1e-8, (method, i, k, c)
        if method == "pipefcg":
            for s, ap in zip(r.trace["S"], AP):
                assert np.linalg.norm(s - ap) <= 1e-10 * np.linalg.norm(ap)


# --- CR and GMRES families --------------------------------------------------
@pytest.mark.parametrize("method", ["gcr", "fgmres", "pipegcr", "pipefgmres"])
def test_linear_pc_minimum_residual(method):
    A, b = _tiny(3, 5, 1.0, seed=6, conv=True)   # nonsymmetric
    Dinv = 1.0 / A.diagonal()
    its = 8
    ref = _min_residual_history(A, b, lambda v: Dinv * v, its)
    r = solve(method, A, jacobi_pc(Dinv), b, rtol=1e-14, maxit=its, nu_max=30)
    tol = 1e-9 if method in ("gcr", "fgmres") else 1e-8
    assert np.allclose(np.array(r.history)[: its + 1], ref, rtol=tol)


def test_pipelined_equals_base_for_linear_pc():
    A, b = _tiny(3, 5, 1.0, seed=7, conv=True)
    B = jacobi_pc(1.0 / A.diagonal())
    for base, pipe in (("gcr", "pipegcr"), ("gcr", "pipegcr_w"), ("fgmres", "pipefgmres")):
        h0 = solve(base, A, B, b, rtol=1e-14, maxit=10, nu_max=30).history
        # sigma defaults to the largest-eigenvalue estimate of A B, as the paper
        # recommends; a shift far from it makes the recurrences unstable
        h1 = solve(pipe, A, B, b, rtol=1e-14, maxit=10, nu_max=30).history
        assert np.allclose(h0[:11], h1[:11], rtol=1e-8), (pipe, h0[:5], h1[:5])


def test_arnoldi_relations():
    A, b = _tiny(3, 5, 1.0, seed=8, conv=True)
    B = make_pc("jacobi_pcg", A, 2)   # nonlinear: U is not M^-1 P
    r = solve("fgmres", A, B, b, rtol=1e-14, maxit=8, nu_max=30, record=True)
    P, U, H = np.array(r.trace["P"]).T, np.array(r.trace["U"]).T, r.trace["H"]
    k = P.shape[1]            # the trace holds p_0..p_{k-1} and k columns of H
    AU = np.array([A.apply(U[:, j]) for j in range(k - 1)]).T
    assert np.linalg.norm(AU - P @ H[:k, : k - 1]) <= 1e-12 * np.linalg.norm(AU)
    assert np.abs(P.T @ P - np.eye(k)).max() <= 1e-12
    sigma = 4.0
    r = solve("pipefgmres", A, B, b, rtol=1e-14, maxit=8, nu_max=30, sigma=sigma, record=True)
    P, U, ZB = (np.array(r.trace[k]).T for k in ("P", "U", "ZB"))
    H = r.trace["H"]
    for j in range(ZB.shape[1]):
        az = A.apply(U[:, j]) - sigma * P[:, j]
        assert np.linalg.norm(ZB[:, j] - az) <= 1e-10 * np.linalg.norm(az)
    k = P.shape[1]
    assert np.abs(P.T @ P - np.eye(k)).max() <= 1e-9
    AU = np.array([A.apply(U[:, j]) for j in range(H.shape[1])]).T
    assert np.linalg.norm(AU[:, : k - 1] - P @ H[:k, : k - 1]) <= 1e-9 * np.linalg.norm(AU)


def test_givens_least_squares_matches_lstsq():
    rng = np.random.default_rng(11)
    for k in (1, 3, 10, 30):
        H = np.triu(rng.standard_normal((k + 1, k)), -1)
        beta = 2.5
        y, res = givens_lstsq(H, beta)
        rhs = np.zeros(k + 1)
        rhs[0] = beta
        ref = np.linalg.lstsq(H, rhs, rcond=None)[0]
        assert np.allclose(y, ref, rtol=1e-10, atol=1e-12)
        assert res == pytest.approx(np.linalg.norm(rhs - H @ ref), rel=1e-9, abs=1e-13)


# --- truncation, restarts, special cases -------------------------------------
def test_truncation_rules_golden():
    g = json.load(open(os.path.join(GOLDEN, "truncation.json")))
    for rule, want in g["expected"].items():
        assert [truncation_nu(rule, j, g["nu_max"]) for j in g["j"]] == want


@pytest.mark.parametrize("rule", ["notay", "modp1"])
def test_alternative_truncations_converge(rule):
    A, b = _tiny(2, 10, 2.0, seed=9)
    r = solve("fcg", A, make_pc("jacobi_pcg", A, 2), b, rtol=1e-8, maxit=300, nu_max=5, truncation=rule)
    assert r.converged


@pytest.mark.parametrize("method", ["fcg", "pipefcg", "gcr", "pipegcr", "pipefgmres"])
def test_forced_breakdown_restarts_and_converges(method):
    A, b = _tiny(2, 10, 1.0, seed=10)
    B = jacobi_pc(1.0 / A.diagonal())
    r0 = solve(method, A, B, b, rtol=1e-8, maxit=300, nu_max=30, sigma=2.0)
    r = solve(method, A, B, b, rtol=1e-8, maxit=300, nu_max=30, sigma=2.0, force_breakdown_at=5)
    assert r.converged and r.restarts == 1
    assert r.history[:5] == r0.history[:5]
    assert len(r.history) == r.iterations + 1


def test_zero_rhs_and_maxit():
    A, b = _tiny()
    B = jacobi_pc(1.0 / A.diagonal())
    r = solve("pipefcg", A, B, np.zeros(A.N), x0=np.ones(A.N))
    assert r.converged and r.iterations == 0 and not np.any(r.x)
    r = solve("pipefcg", A, B, b, rtol=1e-14, maxit=4)
    assert r.status == "maxit" and r.iterations == 4 and len(r.history) == 5


def test_fig1_toy_stagnation():
    g = json.load(open(os.path.join(GOLDEN, "fig1_toy.json")))
    lam, b = gen.toy_diagonal(g["problem"]["n"], g["problem"]["condition_number"])
    xs = b / lam
    lo, hi = g["plateau_band"]
    for eta in g["noise_levels"]:
        err = {}
        for m in ("fcg", "pipefcg_naive", "pipefcg"):
            B = noisy_pc(eta, np.random.default_rng(1))
            r = solve(m, lambda v: lam * v, B, b, rtol=1e-15, maxit=g["check_at_iteration"], nu_max=g["nu_max"])
            err[m] = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
        assert lo * eta <= err["pipefcg_naive"] <= hi * eta, (eta, err)
        assert err["fcg"] < g["converged_error_below"] and err["pipefcg"] < g["converged_error_below"], err


# ---------------------------------------------------------------------------
# natural norm (section 5, implementation remarks)
# ---------------------------------------------------------------------------
def _dense_natural(method, A, Dinv, b, its, nu):
    """sqrt|gamma| recomputed from the true residual of the iterate after each
    of the first ``its`` iterations (separate solves stopped by maxit):
    sqrt(r D^-1 r) for CG types, sqrt|r A D^-1 r| for CR types."""
    out = []
    for i in range(its + 1):
        x = solve(method, A, lambda v: Dinv * v, b, rtol=0.0, maxit=i, nu_max=nu).x
        r = b - A.apply(x)
        g = r @ (Dinv * r) if method in ("fcg", "pipefcg") else r @ A.apply(Dinv * r)
        out.append(math.sqrt(abs(g)))
    return np.array(out)


@pytest.mark.parametrize("method", ["fcg", "pipefcg", "gcr", "pipegcr", "pipegcr_w"])
def test_natural_norm_is_the_b_norm_of_the_true_residual(method):
    conv = method in ("gcr", "pipegcr", "pipegcr_w")
    A, b = _tiny(3, 7, 2.0, seed=5, conv=conv)
    Dinv = 1.0 / A.diagonal()
    ref = solve(method, A, lambda v: Dinv * v, b, rtol=0.0, maxit=8, nu_max=30)
    assert len(ref.natural) == 9
    np.testing.assert_allclose(ref.natural, _dense_natural(method, A, Dinv, b, 8, 30), rtol=1e-8)


@pytest.mark.parametrize("method", ["fcg", "pipefcg", "gcr", "pipegcr"])
def test_natural_norm_stopping(method):
    conv = method in ("gcr", "pipegcr")
    A, b = _tiny(2, 12, 2.0, seed=6, conv=False) if not conv else _tiny(3, 8, 2.0, seed=6, conv=True)
    B = make_pc("jacobi_pcg", A, 2)
    rtol = 1e-6
    full = solve(method, A, B, b, rtol=0.0, maxit=200, nu_max=30)
    nat = np.array(full.natural)
    first = int(np.argmax(nat <= rtol * nat[0]))
    assert nat[first] <= rtol * nat[0] and first > 0
    res = solve(method, A, B, b, rtol=rtol, maxit=200, nu_max=30, norm="natural")
    assert res.converged
    # the accepted iterate meets the tolerance in the natural norm of its true residual
    r = b - A.apply(res.x)
    g = r @ A.apply(B(r)) if conv else B(r) @ r
    assert math.sqrt(abs(g)) <= rtol * nat[0]
    if res.restarts == 0:
        # it stopped at the first recurred crossing
        assert res.iterations == first
        assert np.array_equal(res.natural, nat[:first + 1])
    else:
        # that iterate failed the true-residual check: a gap restart, then a later stop
        assert res.iterations > first
        assert np.array_equal(res.natural[:first + 1], nat[:first + 1])
    # the 2-norm mode logs the same natural norms (FCG/GCR up to the converging iteration)
    two = solve(method, A, B, b, rtol=rtol, maxit=200, nu_max=30)
    n = len(two.natural)
    assert n >= two.iterations and np.array_equal(two.natural, nat[:n])


# ---------------------------------------------------------------------------
# PIPEGCR's stabilised m_i = u_i + B(w_i - r_i) (section 2.2.2, Alg. 11/12)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nu_max", [100, 30])
def test_pipegcr_stabilised_m_with_noisy_pc(nu_max):
    """With B(r) = r + noise (the section 2.2.1 toy), GCR and both PIPEGCR
    forms converge while the same cycle with m_i = B(w_i) stalls near the
    noise level.  For linear B the two m agree exactly, so only a nonlinear B
    shows which one the oracle computes."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_toy.json")))
    lam, b = gen.toy_diagonal(g["problem"]["n"], g["problem"]["condition_number"])
    xs = b / lam
    lo, hi = g["plateau_band"]
    for eta in g["noise_levels"]:
        err = {}
        for m in ("gcr", "pipegcr", "pipegcr_w", "pipegcr_naive", "pipegcr_w_naive"):
            B = noisy_pc(eta, np.random.default_rng(1))
            r = solve(m, lambda v: lam * v, B, b, rtol=1e-15, maxit=g["check_at_iteration"], nu_max=nu_max)
            err[m] = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
        for m in ("pipegcr_naive", "pipegcr_w_naive"):
            assert lo * eta <= err[m] <= hi * eta, (eta, err)
        for m in ("gcr", "pipegcr", "pipegcr_w"):
            assert err[m] < g["converged_error_below"], (eta, err)


def test_pipegcr_stabilised_m_on_a_stencil_with_counter_noise():
    """The same contrast on the unit-scaled 3D Laplacian of the study at scale,
    with the seeded counter-based noise the GPU path also draws."""
    from oracle import CounterNoisyPC
    p = gen.study_problem(3, 10, seed=0)
    A = StencilOperator(3, 10, p.eta, None)
    xs = p.meta["x_star"]
    b = A.apply(xs)
    eta = 1e-2
    err = {}
    for m in ("gcr", "pipegcr", "pipegcr_naive"):
        r = solve(m, A, CounterNoisyPC(eta, 3), b, rtol=1e-12, maxit=150, nu_max=30)
        err[m] = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
    assert err["gcr"] < 1e-9 and err["pipegcr"] < 1e-9, err
    assert 0.3 * eta <= err["pipegcr_naive"] <= 10 * eta, err


def test_naive_and_stabilised_pipegcr_agree_for_linear_pc():
    A, b = _tiny(3, 5, 1.0, seed=7, conv=True)
    B = jacobi_pc(1.0 / A.diagonal())
    for stab, naive in (("pipegcr", "pipegcr_naive"), ("pipegcr_w", "pipegcr_w_naive")):
        h0 = solve(stab, A, B, b, rtol=1e-14, maxit=10, nu_max=30).history
        h1 = solve(naive, A, B, b, rtol=1e-14, maxit=10, nu_max=30).history
        assert np.allclose(h0, h1, rtol=1e-8)


# ---------------------------------------------------------------------------
# PIPEFGMRES shift sigma (sections 4.4 and 5): power-iteration estimate
# ---------------------------------------------------------------------------
def _closed_form_rayleigh(mu, its):
    """Rayleigh quotient after ``its`` power steps on diag(mu) from equal weights:
    v_{its-1} is proportional to mu^(its-1), so R = sum mu^(2 its-1) / sum mu^(2 its-2)."""
    mu = np.asarray(mu, dtype=np.float64)
    s = mu / mu.max()                                    # scaled powers (no overflow)
    return mu.max() * np.sum(s ** (2 * its - 1)) / np.sum(s ** (2 * its - 2))


@pytest.mark.parametrize("its", [1, 2, 10, 25])
def test_estimate_sigma_closed_form_for_diagonal_operators(its):
    from oracle import estimate_sigma
    rng = np.random.default_rng(3)
    lam = np.linspace(1.0, 9.0, 40)
    d = rng.uniform(0.2, 1.5, 40)                        # B = diag(d): A B != A in order and scale
    mu = lam * d
    est = estimate_sigma(lambda v: lam * v, lambda v: d * v, 40, its=its)
    assert est == pytest.approx(_closed_form_rayleigh(mu, its), rel=1e-12)
    # the operator order matters: A alone (no B) gives another value
    assert abs(_closed_form_rayleigh(lam, its) - est) > 1e-3 * est


def test_estimate_sigma_power_iteration_bound():
    """max(mu) - R_k <= (max - min) tan^2(theta_0) (mu_2/mu_1)^(2k-2) for a symmetric
    A B with a simple top eigenvalue, equal start weights (tan^2 theta_0 = N - 1)."""
    from oracle import estimate_sigma
    mu = np.concatenate([np.linspace(0.5, 3.0, 31), [6.0]])
    N = mu.size
    for its in (5, 10, 20):
        est = estimate_sigma(lambda v: mu * v, lambda v: v.copy(), N, its=its)
        gap = (mu.max() - mu.min()) * (N - 1) * (3.0 / 6.0) ** (2 * its - 2)
        assert est <= mu.max() * (1 + 1e-15)
        assert mu.max() - est <= gap, (its, est)
    assert estimate_sigma(lambda v: mu * v, lambda v: v.copy(), N, its=60) == pytest.approx(6.0, rel=1e-12)


def test_estimate_sigma_reaches_largest_eigenvalue_of_jacobi_preconditioned_stencil():
    from oracle import estimate_sigma
    A, _ = _tiny(2, 4, 2.0, seed=1)
    Dinv = 1.0 / A.diagonal()
    ev = np.linalg.eigvals(_dense(A) * Dinv[None, :])    # A D^-1: the right-preconditioned operator
    top = float(np.max(ev.real))
    est = estimate_sigma(A.apply, jacobi_pc(Dinv), A.N, its=400)
    assert est == pytest.approx(top, rel=1e-8)
    # with B = I the same routine finds the top of A's own spectrum instead
    est_a = estimate_sigma(A.apply, lambda v: v.copy(), A.N, its=400)
    assert est_a == pytest.approx(float(np.max(np.linalg.eigvalsh(_dense(A)))), rel=1e-8)
    assert abs(est_a - top) > 1e-2 * top


def test_natural_norm_check_rejects_a_stagnated_iterate():
    """PIPEFCG with the global 2-step inner CG on config 1 stagnates in the true
    residual while its recurred natural norm keeps falling (section 2.2.2: the
    pipelined CG needs a faithful preconditioner).  The natural-norm test must
    not accept such an iterate: every recurred crossing is checked against the
    natural norm of the true residual, and fails, so the solve restarts and
    ends unconverged."""
    p = gen.config_problem("cfg1", seed=0)
    A = StencilOperator(2, 64, p.eta)
    B = make_pc("jacobi_pcg", A, 2)
    r = solve("pipefcg", A, B, p.b, rtol=1e-6, maxit=300, nu_max=30, norm="natural", max_restarts=3)
    assert not r.converged
    assert r.restarts >= 1
    rt = p.b - A.apply(r.x)
    assert math.sqrt(abs(B(rt) @ rt)) > 1e-6 * r.natural[0]
    assert r.true_rel_resid > 1e-3


# ---------------------------------------------------------------------------
# stagnation restart (option stall_window)
# ---------------------------------------------------------------------------
def test_stall_restart_fires_at_the_rule():
    """The restart comes at the first iteration i >= K (since the start) whose
    recurred residual is above half of entry i - K, and not before."""
    p = gen.config_problem("cfg1", seed=0)
    A = StencilOperator(2, 64, p.eta)
    B = make_pc("jacobi_pcg", A, 2)
    h = solve("pipefcg", A, B, p.b, rtol=0.0, maxit=120, nu_max=30).history
    K = 20
    i = next(i for i in range(K, len(h)) if h[i] > 0.5 * h[i - K])
    before = solve("pipefcg", A, B, p.b, rtol=0.0, maxit=i - 1, nu_max=30, stall_window=K)
    at = solve("pipefcg", A, B, p.b, rtol=0.0, maxit=i, nu_max=30, stall_window=K)
    assert before.restarts == 0 and at.restarts == 1
    assert at.history == h[:i + 1]
    # GMRES types ignore the option
    g0 = solve("fgmres", A, jacobi_pc(1.0 / A.diagonal()), p.b, rtol=0.0, maxit=40, nu_max=30)
    g1 = solve("fgmres", A, jacobi_pc(1.0 / A.diagonal()), p.b, rtol=0.0, maxit=40, nu_max=30, stall_window=5)
    assert g0.history == g1.history and g1.restarts == 0


def test_stall_restarts_lift_the_noise_floor():
    """Naive PIPEFCG on the section 2.2.1 toy stalls near the noise level; a
    restart from the current x rebuilds its recurrences there, so with
    stagnation restarts it goes far below the plateau."""
    lam, b = gen.toy_diagonal(100, 5.0)
    xs = b / lam
    err = {}
    for K in (0, 20):
        B = noisy_pc(0.1, np.random.default_rng(1))
        r = solve("pipefcg_naive", lambda v: lam * v, B, b, rtol=1e-15, maxit=200, nu_max=100,
                  stall_window=K, max_restarts=50)
        err[K] = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
    assert err[0] > 1e-4 and err[20] < 1e-7, err
